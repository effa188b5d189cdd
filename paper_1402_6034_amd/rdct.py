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
# RDCT_LIB may name another build of the library (e.g. to compare kernel variants).
LIB_PATH = os.environ.get("RDCT_LIB") or os.path.join(_HERE, "librdct.so")

# rdct_status_t
(OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_HIP, ERR_NO_MEMORY, ERR_BUDGET, ERR_NOT_FOUND, ERR_BUSY,
 ERR_CANCELLED) = range(9)
# rdct_coef_t
COEF_I32, COEF_I16, COEF_F32 = 0, 1, 2
LAYOUT_DEFAULT, LAYOUT_STRIDED, LAYOUT_PER_PLANE = 0, 1, 2
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


class PlaneDesc(ctypes.Structure):
    """rdct_plane_desc_t."""
    _fields_ = [("src", c_void_p), ("width", c_int32), ("height", c_int32),
                ("src_pitch", c_int64), ("sel", Select), ("coef_out", c_void_p),
                ("recon_out", c_void_p), ("recon_pitch", c_int64)]


class Tuning(ctypes.Structure):
    """rdct_tuning_t."""
    _fields_ = [("waves_per_wg", c_int32), ("wgs_per_cu", c_int32), ("use_graph", c_int32),
                ("layout", c_int32), ("xcd_ranges", c_int32), ("strip", c_int32)]


class QualityDesc(ctypes.Structure):
    """rdct_quality_desc_t."""
    _fields_ = [("src", c_void_p), ("width", c_int32), ("height", c_int32),
                ("src_pitch", c_int64)]


def _declare_extra(L):
    """Signatures of the batch and server entry points."""
    P = c_void_p
    L.rdct_batch_plan_create.argtypes = [POINTER(PlaneDesc), c_int32, c_int32, P,
                                         POINTER(Tuning), POINTER(c_void_p)]
    L.rdct_batch_plan_create.restype = c_int32
    L.rdct_batch_plan_create_sweep.argtypes = [POINTER(PlaneDesc), c_int32, c_int32, c_int32, P,
                                               POINTER(Tuning), POINTER(c_void_p)]
    L.rdct_batch_plan_create_sweep.restype = c_int32
    L.rdct_batch_run.argtypes = [P, P]
    L.rdct_batch_run.restype = c_int32
    L.rdct_batch_plan_info.argtypes = [P, POINTER(c_int64), POINTER(c_int32), POINTER(Tuning)]
    L.rdct_batch_plan_set_tuning.argtypes = [P, POINTER(Tuning)]
    L.rdct_batch_plan_set_tuning.restype = c_int32
    L.rdct_batch_plan_info.restype = c_int32
    L.rdct_batch_autotune.argtypes = [P, c_int32, P, POINTER(Tuning)]
    L.rdct_batch_autotune.restype = c_int32
    L.rdct_batch_plan_destroy.argtypes = [P]
    L.rdct_batch_plan_destroy.restype = None
    L.rdct_codec_groups.argtypes = [c_int32, c_int32]
    L.rdct_codec_groups.restype = c_int64
    L.rdct_codec_encode.argtypes = [P, c_int32, c_int32, c_int64, POINTER(Select), P, P, P, P,
                                    c_int64, P]
    L.rdct_codec_encode.restype = c_int32
    L.rdct_codec_pack.argtypes = [P, P, P, c_int32, c_int32, P, P, c_int64, P, P]
    L.rdct_codec_pack.restype = c_int32
    L.rdct_codec_pack_noalloc.argtypes = [P, P, P, c_int32, c_int32, P, P, c_int64, P]
    L.rdct_codec_pack_noalloc.restype = c_int32
    L.rdct_quality_sweep.argtypes = [P, c_int32, c_int32, c_int64, c_int32, c_int32, c_int32, P, P,
                                     P]
    L.rdct_quality_sweep.restype = c_int32
    L.rdct_quality_sse_unit.argtypes = [c_int32]
    L.rdct_quality_sse_unit.restype = c_double
    L.rdct_quality_windows.argtypes = [c_int32, c_int32]
    L.rdct_quality_windows.restype = c_int64
    L.rdct_quality_metrics.argtypes = [P, P, c_int32, c_int32, c_int32, c_int32, P, P]
    L.rdct_quality_metrics.restype = c_int32
    L.rdct_psnr_planes.argtypes = [P, c_int32, c_int32, c_int32, P, P, P, P]
    L.rdct_psnr_planes.restype = c_int32
    L.rdct_psnr_device.argtypes = [P, c_int32, c_int32, c_int32, P, P, P, P]
    L.rdct_psnr_device.restype = c_int32
    L.rdct_codec_unpack_pairs.argtypes = [P, c_int64, P, P]
    L.rdct_codec_unpack_pairs.restype = c_int32
    L.rdct_stream_unit_bytes.argtypes = [c_int32, POINTER(c_int64), POINTER(c_int64)]
    L.rdct_stream_unit_bytes.restype = c_int32
    L.rdct_stream.argtypes = [P, P, c_int64, c_int32, c_int32, c_int32, P]
    L.rdct_stream.restype = c_int32
    L.rdct_quality_plan_create.argtypes = [POINTER(QualityDesc), c_int32, c_int32, c_int32, c_int32,
                                           P, P, POINTER(c_void_p)]
    L.rdct_quality_plan_create.restype = c_int32
    L.rdct_quality_plan_run.argtypes = [P, P]
    L.rdct_quality_plan_run.restype = c_int32
    L.rdct_quality_plan_destroy.argtypes = [P]
    L.rdct_quality_plan_destroy.restype = None
    if hasattr(L, "rdct_server_create"):
        from . import serve as _serve
        _serve.declare(L)


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


# ---------------------------------------------------------------------------
# Batch plans (one persistent launch over many planes)
# ---------------------------------------------------------------------------

def rdct_batch_plan_create(descs, n, coef_type, sse_out, tuning=None):
    h = c_void_p()
    _check(lib().rdct_batch_plan_create(descs, n, coef_type, _ptr(sse_out),
                                        ctypes.byref(tuning) if tuning is not None else None,
                                        ctypes.byref(h)), "rdct_batch_plan_create")
    return h


def rdct_batch_plan_create_sweep(descs, n, r_count, coef_type, sse_out, tuning=None):
    h = c_void_p()
    _check(lib().rdct_batch_plan_create_sweep(descs, n, r_count, coef_type, _ptr(sse_out),
                                              ctypes.byref(tuning) if tuning is not None else None,
                                              ctypes.byref(h)), "rdct_batch_plan_create_sweep")
    return h


def rdct_batch_run(plan, stream=None):
    _check(lib().rdct_batch_run(plan, _stream(stream)), "rdct_batch_run")


def rdct_batch_plan_info(plan):
    nb, ni, t = c_int64(), c_int32(), Tuning()
    _check(lib().rdct_batch_plan_info(plan, ctypes.byref(nb), ctypes.byref(ni), ctypes.byref(t)),
           "rdct_batch_plan_info")
    return nb.value, ni.value, t


def rdct_batch_autotune(plan, reps=5, stream=None):
    t = Tuning()
    _check(lib().rdct_batch_autotune(plan, reps, _stream(stream), ctypes.byref(t)),
           "rdct_batch_autotune")
    return t


def rdct_batch_plan_destroy(plan):
    lib().rdct_batch_plan_destroy(plan)


class BatchPlan:
    """A batch of device planes with their selections; outputs are allocated here
    (coefficients and reconstructions as slices of two flat buffers) and stay
    resident.  `run()` launches the whole batch; `sse` holds one raw error sum
    per plane (see rdct_sse_unit), or with r_count > 1 (a retention sweep over
    r = sel.r .. sel.r + r_count - 1) an (n, r_count) array of them."""

    def __init__(self, planes, sels, coef_type=None, recon=False, tuning=None, device=None,
                 r_count=1):
        if len(planes) != len(sels) or not planes:
            raise ValueError("planes and selections must be non-empty and equal in number")
        dev = planes[0].device if device is None else device
        self.planes, self.sels = list(planes), list(sels)
        self.n = len(planes)
        self.shapes = [tuple(p.shape) for p in planes]
        nbs = [rdct_num_blocks(w, h) for (h, w) in self.shapes]
        self.coef = self.recon = None
        self.coef_views, self.recon_views = [None] * self.n, [None] * self.n
        if coef_type is not None:
            self.coef = torch.empty(sum(nbs) * 64, dtype=_TORCH_DTYPE[coef_type], device=dev)
            off = 0
            for i, nb in enumerate(nbs):
                self.coef_views[i] = self.coef[off:off + nb * 64].view(nb, 64)
                off += nb * 64
        if recon:
            tot = sum(h * w for (h, w) in self.shapes)
            self.recon = torch.empty(tot, dtype=torch.float32, device=dev)
            off = 0
            for i, (h, w) in enumerate(self.shapes):
                self.recon_views[i] = self.recon[off:off + h * w].view(h, w)
                off += h * w
        self.r_count = r_count
        self.sse = torch.zeros(self.n * r_count, dtype=torch.int64, device=dev)
        descs = (PlaneDesc * self.n)()
        for i, (img, sel) in enumerate(zip(self.planes, self.sels)):
            w, h, pitch = _plane_args(img)
            d = descs[i]
            d.src, d.width, d.height, d.src_pitch = img.data_ptr(), w, h, pitch
            d.sel = sel
            d.coef_out = self.coef_views[i].data_ptr() if self.coef is not None else None
            d.recon_out = self.recon_views[i].data_ptr() if recon else None
            d.recon_pitch = w if recon else 0
        self._descs = descs
        self.coef_type = COEF_I32 if coef_type is None else coef_type
        if r_count == 1:
            self.handle = rdct_batch_plan_create(descs, self.n, self.coef_type, self.sse, tuning)
        else:
            self.handle = rdct_batch_plan_create_sweep(descs, self.n, r_count, self.coef_type,
                                                       self.sse, tuning)
            self.sse = self.sse.view(self.n, r_count)
        self.n_blocks, self.n_items, self.tuning = rdct_batch_plan_info(self.handle)

    def run(self, stream=None):
        rdct_batch_run(self.handle, stream)

    def set_tuning(self, tuning):
        _check(lib().rdct_batch_plan_set_tuning(self.handle, ctypes.byref(tuning)),
               "rdct_batch_plan_set_tuning")
        self.tuning = rdct_batch_plan_info(self.handle)[2]

    def autotune(self, reps=5, stream=None):
        self.tuning = rdct_batch_autotune(self.handle, reps, stream)
        return self.tuning

    def close(self):
        if self.handle:
            rdct_batch_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Comparison transforms and quality metrics (rdct_quality_*)
# ---------------------------------------------------------------------------

T_RDCT, T_DCT, T_SDCT, T_RDCT_CEIL, T_RDCT_FLOOR = range(5)


def rdct_quality_sweep(src, width, height, pitch, transform, r_first, r_count, sse_out, uqi_out,
                       stream=None):
    _check(lib().rdct_quality_sweep(_ptr(src), width, height, pitch, transform, r_first, r_count,
                                    _ptr(sse_out), _ptr(uqi_out), _stream(stream)),
           "rdct_quality_sweep")


def rdct_quality_sse_unit(transform):
    return lib().rdct_quality_sse_unit(transform)


def rdct_quality_windows(width, height):
    return lib().rdct_quality_windows(width, height)


def quality_sweep(img: torch.Tensor, transform: int, r_first: int = 1, r_count: int = 45,
                  stream=None):
    """Raw (sse, uqi) int64 tensors of r_count entries for one device plane."""
    w, h, pitch = _plane_args(img)
    sse = torch.empty(r_count, dtype=torch.int64, device=img.device)
    uqi = torch.empty(r_count, dtype=torch.int64, device=img.device)
    rdct_quality_sweep(img, w, h, pitch, transform, r_first, r_count, sse, uqi, stream)
    return sse, uqi


def _host_array(a, dtype):
    """A C-contiguous numpy array of `dtype` (host memory) for a host-array call."""
    import numpy as np
    if isinstance(a, torch.Tensor):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(a, dtype=dtype)


def _np_ptr(a):
    return a.ctypes.data_as(c_void_p)


def rdct_quality_metrics(sse_raw, uqi_raw, transform, width, height):
    """(mse, uqi) float64 numpy arrays from one plane's raw sums (host arrays)."""
    import numpy as np
    sse = _host_array(sse_raw, np.uint64).reshape(-1)
    uqi = _host_array(uqi_raw, np.int64).reshape(-1)
    if sse.size != uqi.size:
        raise ValueError("sse and uqi differ in length")
    mse = np.empty(sse.size, dtype=np.float64)
    mu = np.empty(sse.size, dtype=np.float64)
    _check(lib().rdct_quality_metrics(_np_ptr(sse), _np_ptr(uqi), sse.size, transform, width,
                                      height, _np_ptr(mse), _np_ptr(mu)), "rdct_quality_metrics")
    return mse, mu


def quality_metrics(sse_raw, uqi_raw, transform, height, width):
    """MSE and mean UQI (float64 numpy arrays) from raw sums."""
    return rdct_quality_metrics(sse_raw, uqi_raw, transform, width, height)


def rdct_psnr_planes(sse_raw, r_count, mode, widths, heights, mean=False):
    """PSNR of n planes (n x r_count float64 numpy array) from their raw sums,
    and with mean=True also the r_count means over the planes."""
    import numpy as np
    sse = _host_array(sse_raw, np.uint64).reshape(-1)
    w = _host_array(widths, np.int32)
    h = _host_array(heights, np.int32)
    n = w.size
    if h.size != n or sse.size != n * r_count:
        raise ValueError("sizes and sums do not match")
    out = np.empty(n * r_count, dtype=np.float64)
    avg = np.empty(r_count, dtype=np.float64) if mean else None
    _check(lib().rdct_psnr_planes(_np_ptr(sse), n, r_count, mode, _np_ptr(w), _np_ptr(h),
                                  _np_ptr(out), _np_ptr(avg) if mean else None),
           "rdct_psnr_planes")
    out = out.reshape(n, r_count)
    return (out, avg) if mean else out


def rdct_psnr_device(sse, r_count, mode, pixels, psnr_out, mean_out=None, stream=None):
    """PSNR of n planes on the device: sse (n * r_count int64/uint64 tensor),
    pixels (n int64 tensor of width * height), psnr_out (n * r_count float64
    tensor), optional mean_out (r_count float64 tensor); all on the device."""
    n = pixels.numel()
    if sse.numel() != n * r_count or psnr_out.numel() != n * r_count or \
            (mean_out is not None and mean_out.numel() != r_count):
        raise ValueError("sizes do not match")
    _check(lib().rdct_psnr_device(_ptr(sse), n, r_count, mode, _ptr(pixels), _ptr(psnr_out),
                                  _ptr(mean_out), _stream(stream)), "rdct_psnr_device")


def rdct_codec_unpack_pairs(words):
    """(runs, values) int32 numpy arrays of packed pair words."""
    import numpy as np
    w = _host_array(words, np.int32).reshape(-1)
    runs = np.empty(w.size, dtype=np.int32)
    vals = np.empty(w.size, dtype=np.int32)
    _check(lib().rdct_codec_unpack_pairs(_np_ptr(w), w.size, _np_ptr(runs), _np_ptr(vals)),
           "rdct_codec_unpack_pairs")
    return runs, vals


class QualityPlan:
    """Keep-r sweep of many device planes under one transform in one launch per
    run; sse and uqi are (n, r_count) int64 tensors of raw sums."""

    def __init__(self, planes, transform, r_first=1, r_count=45):
        if not planes:
            raise ValueError("no planes")
        self.planes = list(planes)
        self.n = len(planes)
        self.transform, self.r_first, self.r_count = transform, r_first, r_count
        dev = planes[0].device
        self.sse = torch.empty((self.n, r_count), dtype=torch.int64, device=dev)
        self.uqi = torch.empty((self.n, r_count), dtype=torch.int64, device=dev)
        descs = (QualityDesc * self.n)()
        for i, img in enumerate(self.planes):
            w, h, pitch = _plane_args(img)
            descs[i].src, descs[i].width, descs[i].height, descs[i].src_pitch = (
                img.data_ptr(), w, h, pitch)
        self._descs = descs
        hdl = c_void_p()
        _check(lib().rdct_quality_plan_create(descs, self.n, transform, r_first, r_count,
                                              _ptr(self.sse), _ptr(self.uqi), ctypes.byref(hdl)),
               "rdct_quality_plan_create")
        self.handle = hdl

    def run(self, stream=None):
        _check(lib().rdct_quality_plan_run(self.handle, _stream(stream)), "rdct_quality_plan_run")

    def metrics(self):
        """(mse, uqi) float64 numpy arrays of shape (n, r_count)."""
        import numpy as np
        torch.cuda.synchronize()
        sse, uqi = self.sse.cpu().numpy(), self.uqi.cpu().numpy()
        mse = np.empty(sse.shape)
        mu = np.empty(uqi.shape)
        for i, img in enumerate(self.planes):
            h, w = img.shape
            mse[i], mu[i] = rdct_quality_metrics(sse[i], uqi[i], self.transform, w, h)
        return mse, mu

    def close(self):
        if self.handle:
            lib().rdct_quality_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Codec output (rdct_codec_*)
# ---------------------------------------------------------------------------

def rdct_codec_groups(width, height):
    return lib().rdct_codec_groups(width, height)


class Codec:
    """Device buffers for the codec output of planes of one size: per-block
    pair counts, per-group slots, the packed stream with block offsets, and the
    8-bit reconstruction."""

    def __init__(self, height, width, device="cuda"):
        self.h, self.w = height, width
        self.nb = rdct_num_blocks(width, height)
        self.groups = rdct_codec_groups(width, height)
        self.counts = torch.empty(self.nb, dtype=torch.int16, device=device)
        self.group_pairs = torch.empty(self.groups, dtype=torch.int32, device=device)
        self.slots = torch.empty(self.groups * 4096, dtype=torch.int32, device=device)
        self.offsets = torch.empty(self.nb + 1, dtype=torch.int32, device=device)
        self.packed = torch.empty(self.nb * 64, dtype=torch.int32, device=device)
        self.workspace = torch.empty(self.groups, dtype=torch.int32, device=device)
        self.recon = torch.empty((height, width), dtype=torch.uint8, device=device)

    def encode(self, img, sel, recon=True, stream=None):
        w, h, pitch = _plane_args(img)
        if (h, w) != (self.h, self.w):
            raise ValueError("plane size differs from the codec's")
        _check(lib().rdct_codec_encode(_ptr(img), w, h, pitch, ctypes.byref(sel), _ptr(self.counts),
                                       _ptr(self.group_pairs), _ptr(self.slots),
                                       _ptr(self.recon) if recon else None,
                                       self.recon.stride(0) if recon else 0, _stream(stream)),
               "rdct_codec_encode")

    def pack(self, stream=None):
        _check(lib().rdct_codec_pack(_ptr(self.counts), _ptr(self.group_pairs), _ptr(self.slots),
                                     self.w, self.h, _ptr(self.offsets), _ptr(self.packed),
                                     self.packed.numel(), _ptr(self.workspace), _stream(stream)),
               "rdct_codec_pack")

    def pairs_host(self):
        """Per-block lists of (run, value) from the packed stream."""
        import numpy as np
        torch.cuda.synchronize()
        off = self.offsets.cpu().numpy().astype(np.int64)
        runs, vals = rdct_codec_unpack_pairs(self.packed[:int(off[-1])])
        return [list(zip(runs[off[b]:off[b + 1]].tolist(), vals[off[b]:off[b + 1]].tolist()))
                for b in range(self.nb)]


# ---------------------------------------------------------------------------
# Bandwidth calibration (rdct_stream)
# ---------------------------------------------------------------------------

STREAM_READ, STREAM_WRITE, STREAM_COPY, STREAM_R1W2, STREAM_R1W6 = range(5)


def rdct_stream_unit_bytes(pattern):
    """(read, written) bytes of one unit of `pattern`."""
    rb, wb = c_int64(), c_int64()
    _check(lib().rdct_stream_unit_bytes(pattern, ctypes.byref(rb), ctypes.byref(wb)),
           "rdct_stream_unit_bytes")
    return rb.value, wb.value


def rdct_stream(src, dst, units, pattern, flags=3, wgs_per_cu=0, stream=None):
    """Move `units` units of `pattern` from device tensor src to dst (sizes checked)."""
    rb, wb = rdct_stream_unit_bytes(pattern)
    if src is not None and src.numel() * src.element_size() < units * rb:
        raise ValueError("source smaller than the units read")
    if dst.numel() * dst.element_size() < max(units * wb, 1024):
        raise ValueError("destination smaller than the units written")
    _check(lib().rdct_stream(_ptr(src), _ptr(dst), units, pattern, flags, wgs_per_cu,
                             _stream(stream)), "rdct_stream")
