"""Python binding of librdct (the HIP round-off DCT library).

Thin ctypes layer: the `rdct_*` functions mirror the C-ABI of include/rdct.h one
for one and only marshal arguments; the convenience wrappers below them allocate
output tensors with torch (device memory and streams only) and call the same
entry points.  Every step of the transform runs in the library's HIP kernels.
There is no fallback: if librdct.so is missing or a call fails, an exception is
raised.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_uint16, c_uint64, c_void_p

import torch  # noqa: F401  (loads the HIP runtime that the library shares)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librdct.so")

# rdct_status_t
OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_HIP, ERR_NO_MEMORY, ERR_BUDGET, ERR_NOT_FOUND, ERR_BUSY = range(8)
# rdct_coef_t
COEF_I32, COEF_I16, COEF_F32 = 0, 1, 2
# rdct_sel_mode_t
SEL_NONE, SEL_ZIGZAG, SEL_QUANT = 0, 1, 2

_TORCH_DTYPE = {COEF_I32: torch.int32, COEF_I16: torch.int16, COEF_F32: torch.float32}


class RdctError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = lib().rdct_status_string(status).decode()
        super().__init__(f"{what}: {msg} (status {status})" if what else msg)


class Select(ctypes.Structure):
    """rdct_select_t."""
    _fields_ = [("mode", c_int32), ("r", c_int32), ("quality", c_int32),
                ("level_shift", c_int32), ("qtable", POINTER(c_uint16))]


def select(mode: int = SEL_ZIGZAG, r: int = 64, quality: int = 50, level_shift: int = 0,
           qtable=None) -> Select:
    """Build an rdct_select_t.  `qtable` (64 ints, natural order) is copied into a
    host array kept alive by the returned structure."""
    s = Select(mode=mode, r=r, quality=quality, level_shift=level_shift)
    if qtable is not None:
        arr = (c_uint16 * 64)(*[int(v) for v in list(qtable)])
        s._qt = arr  # keep alive
        s.qtable = ctypes.cast(arr, POINTER(c_uint16))
    return s


_lib = None


def lib() -> ctypes.CDLL:
    """Load librdct.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing; build it with "
                           "`python -m paper_1402_6034_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    sel_p = POINTER(Select)
    L.rdct_forward.argtypes = [c_void_p, c_int32, c_int32, c_int64, sel_p, c_void_p, c_int32, c_void_p]
    L.rdct_inverse.argtypes = [c_void_p, c_int32, c_int32, c_int32, sel_p, c_void_p, c_int64, c_void_p]
    L.rdct_compress_eval.argtypes = [c_void_p, c_int32, c_int32, c_int64, sel_p, c_int32,
                                     c_void_p, c_int32, c_void_p, c_int64, c_void_p, c_void_p]
    for f in ("rdct_forward", "rdct_inverse", "rdct_compress_eval"):
        getattr(L, f).restype = c_int32
    L.rdct_sse_unit.argtypes = [c_int32]
    L.rdct_sse_unit.restype = c_double
    L.rdct_psnr.argtypes = [c_uint64, c_int32, c_int32, c_int32]
    L.rdct_psnr.restype = c_double
    L.rdct_num_blocks.argtypes = [c_int32, c_int32]
    L.rdct_num_blocks.restype = c_int64
    L.rdct_status_string.argtypes = [c_int32]
    L.rdct_status_string.restype = ctypes.c_char_p
    L.rdct_version.argtypes = []
    L.rdct_version.restype = ctypes.c_char_p
    _declare_extra(L)
    _lib = L
    return L


def _declare_extra(L):
    """Signatures of the batch, server and tuning entry points (if present)."""
    try:
        from . import rdct_ext
    except ImportError:  # pragma: no cover
        return
    rdct_ext.declare(L)


def _check(status: int, what: str):
    if status != OK:
        raise RdctError(status, what)


def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream) -> int | None:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---------------------------------------------------------------------------
# Same-name wrappers of the C-ABI (raw pointers / tensors, status checked)
# ---------------------------------------------------------------------------

def rdct_forward(src, width, height, src_pitch, sel: Select, coef, coef_type, stream=None):
    _check(lib().rdct_forward(_ptr(src), width, height, src_pitch, ctypes.byref(sel),
                              _ptr(coef), coef_type, _stream(stream)), "rdct_forward")


def rdct_inverse(coef, coef_type, width, height, sel: Select, dst, dst_pitch, stream=None):
    _check(lib().rdct_inverse(_ptr(coef), coef_type, width, height, ctypes.byref(sel),
                              _ptr(dst), dst_pitch, _stream(stream)), "rdct_inverse")


def rdct_compress_eval(src, width, height, src_pitch, sel: Select, r_count, coef_out, coef_type,
                       recon_out, recon_pitch, sse_out, stream=None):
    _check(lib().rdct_compress_eval(_ptr(src), width, height, src_pitch, ctypes.byref(sel),
                                    r_count, _ptr(coef_out), coef_type, _ptr(recon_out),
                                    recon_pitch, _ptr(sse_out), _stream(stream)),
           "rdct_compress_eval")


def rdct_sse_unit(mode: int) -> float:
    return lib().rdct_sse_unit(mode)


def rdct_psnr(sse: int, mode: int, width: int, height: int) -> float:
    return lib().rdct_psnr(int(sse), mode, width, height)


def rdct_num_blocks(width: int, height: int) -> int:
    return lib().rdct_num_blocks(width, height)


def rdct_version() -> str:
    return lib().rdct_version().decode()


# ---------------------------------------------------------------------------
# Tensor conveniences
# ---------------------------------------------------------------------------

def _plane_args(img: torch.Tensor):
    if img.dtype != torch.uint8 or img.dim() != 2 or not img.is_cuda:
        raise ValueError("expected a 2-D uint8 CUDA tensor")
    if img.stride(1) != 1:
        raise ValueError("plane rows must be contiguous")
    h, w = img.shape
    return w, h, img.stride(0)


def forward(img: torch.Tensor, sel: Select, coef_type: int = COEF_I32, out=None, stream=None):
    """Block-major coefficients (n_blocks, 64) of a plane."""
    w, h, pitch = _plane_args(img)
    nb = rdct_num_blocks(w, h)
    if out is None:
        out = torch.empty((nb, 64), dtype=_TORCH_DTYPE[coef_type], device=img.device)
    rdct_forward(img, w, h, pitch, sel, out, coef_type, stream)
    return out


def inverse(coef: torch.Tensor, height: int, width: int, sel: Select, coef_type: int,
            out=None, stream=None):
    """Float32 plane (height, width) from block-major coefficients."""
    if out is None:
        out = torch.empty((height, width), dtype=torch.float32, device=coef.device)
    rdct_inverse(coef, coef_type, width, height, sel, out, out.stride(0), stream)
    return out


def compress_eval(img: torch.Tensor, sel: Select, r_count: int = 1, coef_type: int | None = None,
                  recon: bool = False, sse=None, coef=None, recon_out=None, stream=None):
    """Fused transform + selection + inverse + squared error.

    Returns (sse, coef, recon): sse is an int64 tensor of r_count raw sums (see
    rdct_sse_unit), coef the block-major coefficients if coef_type is given,
    recon the float32 reconstruction if requested."""
    w, h, pitch = _plane_args(img)
    nb = rdct_num_blocks(w, h)
    if sse is None:
        sse = torch.empty(r_count, dtype=torch.int64, device=img.device)
    if coef_type is not None and coef is None:
        coef = torch.empty((nb, 64), dtype=_TORCH_DTYPE[coef_type], device=img.device)
    if recon and recon_out is None:
        recon_out = torch.empty((h, w), dtype=torch.float32, device=img.device)
    rdct_compress_eval(img, w, h, pitch, sel, r_count, coef,
                       COEF_I32 if coef_type is None else coef_type, recon_out,
                       recon_out.stride(0) if recon_out is not None else 0, sse, stream)
    return sse, coef, recon_out


def psnr_from_sse(sse_raw: int, mode: int, height: int, width: int) -> float:
    return rdct_psnr(int(sse_raw), mode, width, height)
