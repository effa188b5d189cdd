#!/usr/bin/env python3
"""Throughput benchmark of the round-off DCT hot path on one MI355X.

Prints one JSON line.  `--workload` selects the input set; the default is the
ragged batch (1000 planes, forward + quantise + inverse + PSNR).
Timed region: `--steps` passes of the whole path over one batch whose inputs
are already resident in device memory, bracketed by device synchronisations.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "RDCT fwd+inv Mblocks/s & % HBM peak; served p50/p99 latency vs plain"
HBM_PEAK_GBS = 8000.0
N_CU = 256
CLOCK_GHZ = 2.4
# Integer VALU peak: 256 CUs x 64 lanes x 2.4 GHz (one 32-bit op per lane per clock).
ALU_PEAK_TOPS = N_CU * 64 * CLOCK_GHZ / 1000.0
# Published float64 vector peak of MI355X (an FMA counts as two operations).
FP64_PEAK_TFLOPS = 78.6


# Sources that decide each workload's dominant kernel and its launch: a profile
# record counts only while the code of its workload's files is unchanged.
_CSRC = "paper_1402_6034_amd/csrc/"
_COMMON = (_CSRC + "rdct_internal.h", _CSRC + "rdct_tables.h", "include/rdct.h",
           "paper_1402_6034_amd/build.py")
KERNEL_SOURCES = {
    "ragged": (_CSRC + "rdct_kernels.hip", _CSRC + "rdct_device.h", _CSRC + "rdct_batch.cpp"),
    "sweep": (_CSRC + "rdct_kernels.hip", _CSRC + "rdct_device.h", _CSRC + "rdct_batch.cpp"),
    "frame": (_CSRC + "rdct_kernels.hip", _CSRC + "rdct_device.h", _CSRC + "rdct_api.cpp"),
    "quality": (_CSRC + "rdct_quality.hip", _CSRC + "rdct_quality_api.cpp",
                _CSRC + "rdct_transforms.cpp"),
    "codec": (_CSRC + "rdct_codec.hip", _CSRC + "rdct_device.h", _CSRC + "rdct_codec_api.cpp"),
    "inverse": (_CSRC + "rdct_kernels.hip", _CSRC + "rdct_device.h", _CSRC + "rdct_api.cpp"),
    "single": (_CSRC + "rdct_kernels.hip", _CSRC + "rdct_device.h", _CSRC + "rdct_api.cpp"),
    "stream": (_CSRC + "rdct_stream.hip", _CSRC + "rdct_device.h"),
}


def _code_only(text):
    """C/C++ source without comments and blank lines, so that editing a comment
    leaves a record standing (string and character literals are kept whole)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    lines = ("".join(out)).split("\n")
    return "\n".join(ln.rstrip() for ln in lines if ln.strip())


def kernel_source_hash(workload):
    """sha256 over the code (comments and blank lines removed) of the files that
    decide the workload's dominant kernel and its launch, and over the compiler
    flags of the build (its HIP_FLAGS list, not the rest of the build script)."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[workload] + _COMMON:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            text = f.read()
        if rel.endswith(".py"):
            text = text[text.index("HIP_FLAGS = ["):]
            text = text[:text.index("]") + 1]
        else:
            text = _code_only(text)
        h.update(text.encode())
    return h.hexdigest()


def _record(workload, kind):
    """Fields of profiles/<workload>_<kind>.txt, or None when there is no record
    or it was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{workload}_{kind}.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    return rec if rec.get("source_sha256") == kernel_source_hash(workload) else None


def valu_record(workload):
    """VALU wave instructions per launch of the workload's dominant kernel, from
    the counter record profiles/<workload>_valu.txt (SQ_INSTS_VALU), or None."""
    rec = _record(workload, "valu")
    try:
        return int(rec["valu_wave_instructions_per_launch"]) if rec else None
    except (KeyError, ValueError):
        return None


def geometry_tag(cfg):
    """Launch geometry of a batch plan as written in its profile records, from
    the plan's config(); None for workloads without one."""
    if "layout" not in cfg:
        return None
    return (f"{cfg['layout']} {cfg['waves_per_wg']} waves/WG x {cfg['wgs_per_cu']} WGs/CU "
            f"xcd_ranges {int(cfg['xcd_ranges'])} strip {cfg.get('strip', 1)}")


def traffic_record(workload, geometry=None):
    """HBM bytes per launch of the workload's dominant kernel, from the counter
    records profiles/<workload>_traffic*.txt (FETCH_SIZE and WRITE_SIZE scaled
    by a device copy of known size; batch plans keep one record per profiled
    launch geometry, since the order in which work items meet the L2s changes
    the bytes read).  None when no record was taken on the current kernel
    sources (and, for batch plans, at the geometry the plan runs)."""
    import glob
    rec = None
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", f"{workload}_traffic*.txt"))):
        r = {}
        with open(path) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    r[k.strip()] = v.strip()
        if r.get("source_sha256") != kernel_source_hash(workload):
            continue
        if geometry is not None and r.get("geometry") != geometry:
            continue
        rec = r
        break
    if rec is None:
        return None
    try:
        out = {"bytes": int(rec["traffic_bytes_per_launch"]),
               "read": int(rec["read_bytes_per_launch"]),
               "write": int(rec["write_bytes_per_launch"])}
    except (KeyError, ValueError):
        return None
    try:
        out["profiler_us"] = float(rec["profiler_kernel_average_us"])
    except (KeyError, ValueError):
        pass
    return out


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def event_time_ms(fn, reps):
    """Average duration of one launch fn(i): HIP events on torch's current stream
    (the stream every library call here is issued on) bracket `reps` launches
    issued back to back, so per-launch event overhead does not count."""
    import torch
    fn(0)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for i in range(reps):
        fn(i)
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / reps


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

class FrameQuant:
    """One 8192 x 8192 luma frame: forward + S-scaled quality-50 quantisation to
    int16 (HBM-bound streaming case).  Six buffer sets (1.2 GB) rotate so the
    256 MB last-level cache never holds the next launch's data."""
    name = "frame-8192-q50-fwd"
    workload_key = "frame"
    dtype = "int16+f64"
    sets = 6

    def __init__(self, size=8192):
        import torch
        from paper_1402_6034_amd import rdct as R, synth
        self.R = R
        self.size = size
        self.nb = (size // 8) ** 2
        log(f"[bench] rendering {size}x{size} frame")
        frame = synth.render(0, size, size, device="cuda")
        self.frames = [frame] + [frame.clone() for _ in range(self.sets - 1)]
        self.coefs = [torch.empty((self.nb, 64), dtype=torch.int16, device="cuda")
                      for _ in range(self.sets)]
        self.sel = R.select(R.SEL_QUANT, quality=50, level_shift=128)
        self.i = 0

    def launch(self, i=None):
        k = self.i if i is None else i % self.sets
        self.R.forward(self.frames[k], self.sel, self.R.COEF_I16, out=self.coefs[k])
        self.i = (self.i + 1) % self.sets

    def step(self):
        self.launch()

    blocks_per_step = property(lambda self: self.nb)
    bytes_per_block = 64 + 128
    kernel_launch = launch

    def config(self):
        return {"workload": self.name, "frame": [self.size, self.size], "blocks": self.nb,
                "quality": 50, "coef": "int16", "level_shift": 128}

    def cpu_baseline(self, budget_s):
        import numpy as np
        import oracle as O
        img = self.frames[0].cpu().numpy()
        rows = 512  # a band of 64 block rows (65,536 blocks)
        t0 = time.perf_counter()
        n = 0
        qt = O.quant_table(50)
        while True:
            band = img[(n * rows) % self.size:(n * rows) % self.size + rows]
            O.quantize(O.forward_image(band, 128), qt)
            n += 1
            if time.perf_counter() - t0 > budget_s:
                break
        dt = time.perf_counter() - t0
        blocks = n * (rows // 8) * (self.size // 8)
        return {"value": blocks / dt / 1e6, "unit": "Mblocks/s", "cores": _oracle_threads(),
                "kind": "oracle",
                "sample": f"{n} bands of {rows}x{self.size} px ({blocks} blocks) of the frame, "
                          "forward + exact quantisation"}


class InverseFrame:
    """rdct_inverse of one 8192 x 8192 frame's quality-50 quantised int16
    coefficients back to float32 pixels (float64 dequantisation and transposed
    transform, level shift added back).  Four buffer sets rotate so the 256 MB
    last-level cache never holds the next launch's data."""
    name = "inverse-frame-8192-q50-i16-f32"
    workload_key = "inverse"
    dtype = "int16+f64"
    sets = 4

    def __init__(self, size=8192):
        import torch
        from paper_1402_6034_amd import rdct as R, synth
        self.R = R
        self.size = size
        self.nb = (size // 8) ** 2
        log(f"[bench] rendering {size}x{size} frame")
        frame = synth.render(0, size, size, device="cuda")
        self.sel = R.select(R.SEL_QUANT, quality=50, level_shift=128)
        q = torch.empty((self.nb, 64), dtype=torch.int16, device="cuda")
        R.forward(frame, self.sel, R.COEF_I16, out=q)
        del frame
        self.coefs = [q] + [q.clone() for _ in range(self.sets - 1)]
        self.recons = [torch.empty((size, size), dtype=torch.float32, device="cuda")
                       for _ in range(self.sets)]
        self.i = 0

    def launch(self, i=None):
        k = self.i if i is None else i % self.sets
        self.R.inverse(self.coefs[k], self.size, self.size, self.sel, self.R.COEF_I16,
                       out=self.recons[k])
        self.i = (self.i + 1) % self.sets

    kernel_launch = launch

    def step(self):
        self.launch()

    blocks_per_step = property(lambda self: self.nb)
    bytes_per_block = 128 + 256

    def config(self):
        return {"workload": self.name, "frame": [self.size, self.size], "blocks": self.nb,
                "quality": 50, "coef": "int16", "recon": "float32", "level_shift": 128}

    def cpu_baseline(self, budget_s):
        import numpy as np
        import oracle as O
        q = self.coefs[0].cpu().numpy().astype(np.int64).reshape(self.size // 8, self.size // 8, 8, 8)
        qt = O.quant_table(50)
        rows = 64  # block rows per band
        t0 = time.perf_counter()
        n = 0
        while time.perf_counter() - t0 < budget_s:
            band = q[(n * rows) % (self.size // 8):][:rows]
            O.inverse_orth(O.dequantize(band, qt))
            n += 1
        dt = time.perf_counter() - t0
        blocks = n * rows * (self.size // 8)
        return {"value": blocks / dt / 1e6, "unit": "Mblocks/s", "cores": _oracle_threads(),
                "kind": "oracle",
                "sample": f"{n} bands of {rows} block rows ({blocks} blocks): dequantise and "
                          "float64 inverse"}


class ResultPipe:
    """Read-back of a step's results (the PSNR values formed on the device) for
    steps run two deep.  Step k writes its results into device buffer k & 1
    (buffer(slot) first makes the launch stream wait until that buffer's last
    transfer is done); submit(slot) has a side stream copy it into pinned host
    buffer `slot`, so the transfer overlaps the next step's kernels; take(slot)
    waits for that transfer and returns the values.  (A copy to the host behind
    the kernel on the launch stream measured 86 to 335 us per step on the
    256-plane sweep, against 97 us on a side stream.)"""

    def __init__(self, n, dtype):
        import torch
        self.dev = [torch.empty(n, dtype=dtype, device="cuda") for _ in range(2)]
        self.host = [torch.empty(n, dtype=dtype, pin_memory=True) for _ in range(2)]
        self.side = torch.cuda.Stream()
        self.ready = [torch.cuda.Event() for _ in range(2)]
        self.copied = [torch.cuda.Event() for _ in range(2)]
        self.used = [False, False]

    def buffer(self, slot):
        import torch
        if self.used[slot]:
            torch.cuda.current_stream().wait_event(self.copied[slot])
        return self.dev[slot]

    def submit(self, slot):
        import torch
        self.ready[slot].record(torch.cuda.current_stream())
        self.side.wait_event(self.ready[slot])
        with torch.cuda.stream(self.side):
            self.host[slot].copy_(self.dev[slot], non_blocking=True)
            self.copied[slot].record(self.side)
        self.used[slot] = True

    def take(self, slot):
        self.copied[slot].synchronize()
        return self.host[slot].numpy()


def seeded_planes(n, size, planes_cache=None):
    """Planes 0..n-1 of size x size from the synthetic generator, on the device.
    With planes_cache, loaded from (or first written to) that .npy file, so a
    profiled run issues no rendering kernels."""
    import numpy as np
    import torch
    from paper_1402_6034_amd import synth
    if planes_cache and os.path.exists(planes_cache):
        log(f"[bench] loading {n} planes from {planes_cache}")
        arr = np.load(planes_cache)
        return [torch.from_numpy(arr[s]).cuda() for s in range(n)]
    log(f"[bench] rendering {n} planes {size}x{size}")
    imgs = [synth.render(s, size, size, device="cuda") for s in range(n)]
    if planes_cache:
        np.save(planes_cache, np.stack([im.cpu().numpy() for im in imgs]))
    return imgs



# rdct_layout_t of a batch plan's tuning.
LAYOUT_NAME = {1: "strided", 2: "per-plane"}

class RetentionSweep:
    """256 planes of 512 x 512, seeds 0..255: forward to int32 coefficients and
    the retention error of every plane for r = 1..45 (exact integer SSE from
    coefficient energies, then PSNR): one persistent batch launch per step.
    `plain()` times the same work as one rdct_compress_eval launch per plane."""
    name = "sweep-256x512x512-r1-45"
    workload_key = "sweep"
    dtype = "int32+int64"

    def __init__(self, n=256, size=512, autotune=True, planes_cache=None):
        from paper_1402_6034_amd import rdct as R
        self.R = R
        self.n, self.size = n, size
        self.imgs = seeded_planes(n, size, planes_cache)
        self.sel = R.select(R.SEL_ZIGZAG, r=1)
        self.plan = R.BatchPlan(self.imgs, [self.sel] * n, R.COEF_I32, recon=False, r_count=45)
        if autotune:
            t = self.plan.autotune(reps=5)
            log(f"[bench] autotuned: {LAYOUT_NAME[t.layout]}, waves/wg {t.waves_per_wg}, "
                f"wg/cu {t.wgs_per_cu}, strip {t.strip}")
        self.nb1 = (size // 8) ** 2
        self.psnr = None

    def launch(self, i=0):
        self.plan.run()

    kernel_launch = launch

    def submit(self, slot):
        """Enqueue one step: the plan run, the PSNR of its sums on the device
        (per plane and r, and the average over planes at every r) and the copy
        of those decibels to the host."""
        import torch
        if getattr(self, "pipe", None) is None:
            self.pixels = torch.full((self.n,), self.size * self.size, dtype=torch.int64,
                                     device="cuda")
            self.pipe = ResultPipe(self.n * 45 + 45, torch.float64)
            self.views = [(d[:self.n * 45], d[self.n * 45:]) for d in self.pipe.dev]
        self.pipe.buffer(slot)
        self.plan.run()
        db, mean = self.views[slot]
        self.R.rdct_psnr_device(self.plan.sse, 45, self.R.SEL_ZIGZAG, self.pixels, db, mean)
        self.pipe.submit(slot)

    def finish(self, slot):
        """Wait for the step in `slot`: per-plane PSNR and the average PSNR over
        the planes for every r (Section 3's curve)."""
        db = self.pipe.take(slot)
        self.psnr = db[:self.n * 45].reshape(self.n, 45)
        self.avg_psnr = db[self.n * 45:]

    def report(self):
        """Average PSNR over the planes at r = 1..45 (the paper's Fig. 3 measure,
        on the synthetic planes)."""
        if getattr(self, "avg_psnr", None) is None:
            return None
        return {"psnr_curve": {"avg_psnr_db_r1_45": [round(float(v), 4) for v in self.avg_psnr],
                               "planes": self.n, "parity_with_paper": "unpinned"}}

    def step(self):
        self.submit(0)
        self.finish(0)

    blocks_per_step = property(lambda self: self.n * self.nb1)
    bytes_per_block = 64 + 256

    def config(self):
        t = self.plan.tuning
        return {"workload": self.name, "planes": self.n, "plane": [self.size, self.size],
                "r": [1, 45], "coef": "int32", "layout": LAYOUT_NAME[t.layout],
                "kernel_launches_per_step": 1 if t.layout == 2 else 2,
                "waves_per_wg": t.waves_per_wg, "wgs_per_cu": t.wgs_per_cu,
                "xcd_ranges": bool(t.xcd_ranges), "strip": t.strip, "graph": bool(t.use_graph)}

    def plain(self, steps=3):
        """The same sweep as one rdct_compress_eval launch per plane."""
        import torch
        R = self.R
        sse = torch.empty((self.n, 45), dtype=torch.int64, device="cuda")
        coef = torch.empty((self.n, self.nb1, 64), dtype=torch.int32, device="cuda")

        def one(k):
            R.compress_eval(self.imgs[k], self.sel, 45, R.COEF_I32, sse=sse[k], coef=coef[k])

        def once():
            for k in range(self.n):
                one(k)
            sse.cpu()
        once()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            once()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        k_ms = event_time_ms(lambda i: one(i % self.n), 64)
        same = bool(torch.equal(sse, self.plan.sse)) and bool(torch.equal(coef.view(-1),
                                                                           self.plan.coef))
        return {"value": round(self.blocks_per_step / (ms * 1e-3) / 1e6, 3), "unit": "Mblocks/s",
                "ms_per_step": round(ms, 4), "launches_per_step": self.n,
                "kernel_ms_per_plane": round(k_ms, 5), "identical_output": same}

    def cpu_baseline(self, budget_s):
        import oracle as O
        t0 = time.perf_counter()
        n = 0
        while True:
            O.retention_eval(self.imgs[n % self.n].cpu().numpy(), range(1, 46))
            n += 1
            if time.perf_counter() - t0 > budget_s:
                break
        dt = time.perf_counter() - t0
        return {"value": n * self.nb1 / dt / 1e6, "unit": "Mblocks/s", "cores": _oracle_threads(),
                "kind": "oracle",
                "sample": f"{n} of the 256 planes, r = 1..45 each (inverse per r, exact SSE)"}


class CodecFrame:
    """Codec output of one 8192 x 8192 frame at quality 50: transform, exact
    quantisation, zig-zag run-length pairs of every block and the 8-bit
    reconstruction (encode), then the packed stream with block offsets (pack).
    Four buffer sets rotate so the 256 MB last-level cache never holds the next
    launch's data."""
    name = "codec-frame-8192-q50-rle-u8"
    workload_key = "codec"
    dtype = "int32+f64"
    sets = 4

    def __init__(self, size=8192):
        from paper_1402_6034_amd import rdct as R, synth
        self.R = R
        self.size = size
        self.nb = (size // 8) ** 2
        log(f"[bench] rendering {size}x{size} frame")
        frame = synth.render(0, size, size, device="cuda")
        self.frames = [frame] + [frame.clone() for _ in range(self.sets - 1)]
        self.codecs = [R.Codec(size, size, "cuda") for _ in range(self.sets)]
        self.sel = R.select(R.SEL_QUANT, quality=50, level_shift=128)
        self.i = 0
        self.launch(0)
        self.codecs[0].pack()
        import torch
        torch.cuda.synchronize()
        self.pairs = int(self.codecs[0].offsets[-1])
        log(f"[bench] {self.pairs} pairs ({self.pairs / self.nb:.2f} per block)")

    def launch(self, i=None):
        k = self.i if i is None else i % self.sets
        self.codecs[k].encode(self.frames[k], self.sel)
        self.i = (self.i + 1) % self.sets

    kernel_launch = launch

    def step(self):
        k = self.i
        self.launch()
        self.codecs[k].pack()

    blocks_per_step = property(lambda self: self.nb)
    # encode: 64 B of pixels in, 64 B of 8-bit pixels, a 2-byte count and 4 B per
    # pair out (the dominant kernel); the pairs per block are measured.
    bytes_per_block = property(lambda self: 64 + 64 + 2 + 4 * self.pairs / self.nb)

    def config(self):
        return {"workload": self.name, "frame": [self.size, self.size], "blocks": self.nb,
                "quality": 50, "level_shift": 128, "pairs": self.pairs,
                "outputs": ["rle_pairs_int32", "offsets_uint32", "recon_u8"]}

    def cpu_baseline(self, budget_s):
        import oracle as O
        img = self.frames[0].cpu().numpy()
        t0 = time.perf_counter()
        n, rows = 0, 64
        while True:
            y0 = (n * rows) % self.size
            O.codec_encode(img[y0:y0 + rows], "quant", quality=50, level_shift=128)
            n += 1
            if time.perf_counter() - t0 > budget_s:
                break
        dt = time.perf_counter() - t0
        blocks = n * (rows // 8) * (self.size // 8)
        return {"value": blocks / dt / 1e6, "unit": "Mblocks/s", "cores": _oracle_threads(),
                "kind": "oracle",
                "sample": f"{n} bands of {rows}x{self.size} px ({blocks} blocks): quantise, "
                          "run-length pairs, 8-bit reconstruction"}


class QualitySweep:
    """The comparison of Section 3 at the paper's image size: 256 planes of
    512 x 512, keep-r sweep over r = 1..45 under the exact DCT, the round-off
    approximation and the signed DCT, scored per plane by MSE and by the mean
    UQI over 8x8 windows; averaged over planes and given as the APE of each
    approximation relative to the DCT.  One launch per transform (a device list
    of 32 x 32 window tiles over all planes)."""
    name = "quality-256x512x512-dct-rdct-sdct-r1-45"
    workload_key = "quality"
    dtype = "f64"
    roofline_kind = "alu"
    # Algorithmic float64 operations per pixel and r: reconstruction update 2
    # (one FMA), squared error 3, the three sliding window sums 2 products + 12
    # adds, the index formula and its two divisions about 14, and the forward
    # transform (2048 per block over 45 values of r) about 1 -> 34.
    flops_per_pixel_r = 34

    def __init__(self, n=256, size=512, r_count=45, planes_cache=None):
        from paper_1402_6034_amd import rdct as R
        self.R = R
        self.n, self.size, self.r_count = n, size, r_count
        self.imgs = seeded_planes(n, size, planes_cache)
        self.transforms = [R.T_DCT, R.T_RDCT, R.T_SDCT]
        self.plans = [R.QualityPlan(self.imgs, t, 1, r_count) for t in self.transforms]
        self.nb1 = (size // 8) ** 2
        self.summary = None

    def launch(self, i=0):
        self.plans[i % len(self.plans)].run()

    kernel_launch = launch

    def step(self):
        import numpy as np
        for p in self.plans:
            p.run()
        mets = [p.metrics() for p in self.plans]          # (mse, uqi), each (n, r)
        mse = [m[0].mean(axis=0) for m in mets]
        uqi = [m[1].mean(axis=0) for m in mets]
        ape = {}
        for j, nm in ((1, "rdct"), (2, "sdct")):
            ape[nm] = {"mse": (100 * np.abs(mse[j] - mse[0]) / mse[0]).tolist(),
                       "uqi": (100 * np.abs(uqi[j] - uqi[0]) / uqi[0]).tolist()}
        self.summary = {"avg_mse": {"dct": mse[0].tolist(), "rdct": mse[1].tolist(),
                                    "sdct": mse[2].tolist()},
                        "avg_uqi": {"dct": uqi[0].tolist(), "rdct": uqi[1].tolist(),
                                    "sdct": uqi[2].tolist()},
                        "ape": ape}

    blocks_per_step = property(lambda self: 3 * self.n * self.nb1)
    # one launch covers one transform over every plane
    flops_per_launch = property(lambda self: self.n * self.size * self.size * self.r_count
                                * self.flops_per_pixel_r)

    def config(self):
        return {"workload": self.name, "planes": self.n, "plane": [self.size, self.size],
                "r": [1, self.r_count], "transforms": ["dct", "rdct", "sdct"],
                "metrics": ["mse", "uqi_8x8"], "launches_per_step": 3}

    def report(self):
        """APE at a few r (the full curves are in the summary)."""
        if not self.summary:
            return None
        pick = [1, 5, 10, 20, 30, 45]
        out = {}
        for nm, a in self.summary["ape"].items():
            out[nm] = {k: {str(r): round(a[k][r - 1], 4) for r in pick} for k in ("mse", "uqi")}
        return {"quality": {"ape_percent": out}}

    def cpu_baseline(self, budget_s):
        import oracle as O
        names = ["dct", "rdct", "sdct"]
        t0 = time.perf_counter()
        n = 0
        while True:
            img = self.imgs[n % self.n].cpu().numpy()
            for nm in names:
                O.quality_eval(img, nm, range(1, self.r_count + 1))
            n += 1
            if time.perf_counter() - t0 > budget_s:
                break
        dt = time.perf_counter() - t0
        return {"value": 3 * n * self.nb1 / dt / 1e6, "unit": "Mblocks/s",
                "cores": _oracle_threads(), "kind": "oracle",
                "sample": f"{n} of the 256 planes x 3 transforms, r = 1..{self.r_count} "
                          "(reconstruction, SSE and 8x8-window UQI per r)"}


class RaggedBatch:
    """1000 planes, width and height independently log-uniform in [64, 4096]
    (multiples of 8), quality uniform in 10..90: forward + S-scaled quantisation
    + inverse + per-plane PSNR in one persistent launch over a device-side block
    work list (hipGraph replay, autotuned geometry); int16 coefficients and the
    float32 reconstruction are written to HBM."""
    name = "ragged-1000-logU64-4096-q10-90"
    workload_key = "ragged"
    dtype = "int16+f64"

    def __init__(self, n=1000, planes_cache=None, autotune=True):
        import numpy as np
        import torch
        from paper_1402_6034_amd import rdct as R, synth
        self.R = R
        self.items = synth.ragged_batch(0, n)
        if planes_cache and os.path.exists(planes_cache):
            log(f"[bench] loading {n} ragged planes from {planes_cache}")
            flat = np.load(planes_cache, mmap_mode="r")
            self.imgs, off = [], 0
            for it in self.items:
                k = it.height * it.width
                self.imgs.append(torch.from_numpy(np.array(flat[off:off + k]).reshape(it.height, it.width)).cuda())
                off += k
        else:
            log(f"[bench] rendering {n} ragged planes")
            self.imgs = [synth.render(it.seed, it.height, it.width, device="cuda") for it in self.items]
            if planes_cache:
                np.save(planes_cache, np.concatenate([im.cpu().numpy().reshape(-1) for im in self.imgs]))
        torch.cuda.synchronize()
        self.sels = [R.select(R.SEL_QUANT, quality=it.quality, level_shift=128) for it in self.items]
        self.plan = R.BatchPlan(self.imgs, self.sels, R.COEF_I16, recon=True)
        self.nb = self.plan.n_blocks
        log(f"[bench] plan: {self.nb} blocks in {self.plan.n_items} work items")
        if autotune:
            t = self.plan.autotune(reps=10)
            log(f"[bench] tuned geometry: {LAYOUT_NAME[t.layout]}, {t.waves_per_wg} waves/WG x "
                f"{t.wgs_per_cu} WGs/CU, XCD ranges {t.xcd_ranges}, strip {t.strip}")
        self.px = sum(it.height * it.width for it in self.items)
        self.psnr = None

    def launch(self, i=0):
        self.plan.run()

    kernel_launch = launch

    def submit(self, slot):
        """Enqueue one step: the plan run, the per-plane PSNR of its sums on the
        device and the copy of those decibels to the host."""
        import torch
        if getattr(self, "pipe", None) is None:
            self.pixels = torch.tensor([it.width * it.height for it in self.items],
                                       dtype=torch.int64, device="cuda")
            self.pipe = ResultPipe(len(self.items), torch.float64)
        db = self.pipe.buffer(slot)
        self.plan.run()
        self.R.rdct_psnr_device(self.plan.sse, 1, self.R.SEL_QUANT, self.pixels, db)
        self.pipe.submit(slot)

    def finish(self, slot):
        """Wait for the step in `slot`: per-plane PSNR."""
        self.psnr = self.pipe.take(slot)

    def step(self):
        self.submit(0)
        self.finish(0)

    blocks_per_step = property(lambda self: self.nb)
    bytes_per_block = 64 + 128 + 256

    def config(self):
        t = self.plan.tuning
        return {"workload": self.name, "planes": len(self.items), "blocks": self.nb,
                "pixels": self.px, "coef": "int16", "recon": "float32", "level_shift": 128,
                "layout": LAYOUT_NAME[t.layout], "waves_per_wg": t.waves_per_wg,
                "wgs_per_cu": t.wgs_per_cu, "xcd_ranges": bool(t.xcd_ranges), "strip": t.strip,
                "graph": bool(t.use_graph)}

    def tuning_table(self, reps=10):
        """Every geometry the autotuner considers (the strided ones with strips of
        1, 2, 4 and 8 items, and with one item also in the hardware's workgroup
        order), plus hipGraph replay of each, timed on this plan (HIP events over
        `reps` back-to-back runs, median of three rounds); the plan keeps its
        tuned geometry afterwards."""
        R = self.R
        keep = self.plan.tuning
        cands = []
        for wpg in (1, 2, 4):
            for waves in (2, 4, 8, 12, 16):
                if waves % wpg == 0:
                    cands.append((wpg, waves // wpg, R.LAYOUT_STRIDED, 0, 1))
                    for strip in (1, 2, 4, 8):
                        cands.append((wpg, waves // wpg, R.LAYOUT_STRIDED, 1, strip))
            cands.append((wpg, 1, R.LAYOUT_PER_PLANE, 0, 1))
        rows = []
        for wpg, wpc, lay, xcd, strip in cands:
            for graph in (0, 1):
                self.plan.set_tuning(R.Tuning(wpg, wpc, graph, lay, xcd, strip))
                ms = sorted(event_time_ms(lambda i: self.plan.run(), reps) for _ in range(3))[1]
                rows.append({"layout": LAYOUT_NAME[lay], "waves_per_wg": wpg, "wgs_per_cu": wpc,
                             "xcd_ranges": bool(xcd), "strip": strip, "graph": bool(graph),
                             "ms": round(ms, 4)})
        self.plan.set_tuning(keep)
        return sorted(rows, key=lambda r: r["ms"])

    def plain(self, steps=2):
        """Same planes through the plain path: one rdct_compress_eval launch per plane."""
        import torch
        R = self.R
        outs = [(torch.empty((R.rdct_num_blocks(im.shape[1], im.shape[0]), 64), dtype=torch.int16,
                             device="cuda"), torch.empty(im.shape, dtype=torch.float32, device="cuda"))
                for im in self.imgs]
        sse = torch.empty((len(self.imgs), 1), dtype=torch.int64, device="cuda")

        def once():
            for k, (im, sel) in enumerate(zip(self.imgs, self.sels)):
                R.compress_eval(im, sel, 1, R.COEF_I16, True, sse=sse[k], coef=outs[k][0],
                                recon_out=outs[k][1])
            sse.cpu()
        once()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            once()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        same = bool(torch.equal(sse[:, 0], self.plan.sse))
        return {"value": round(self.nb / (ms * 1e-3) / 1e6, 3), "unit": "Mblocks/s",
                "ms_per_step": round(ms, 4), "launches_per_step": 2 * len(self.imgs),
                "identical_sse": same}

    def cpu_baseline(self, budget_s):
        """The oracle on planes taken in a seeded random order (so the sample has
        the batch's size mix) until the budget is spent; host copies are made
        before the clock starts."""
        import numpy as np
        import oracle as O
        order = np.random.default_rng(1).permutation(len(self.items))
        t0 = time.perf_counter()
        blocks = n = 0
        spent = 0.0
        while spent < budget_s and n < len(order):
            k = int(order[n])
            it = self.items[k]
            img = self.imgs[k].cpu().numpy()
            t1 = time.perf_counter()
            O.quant_eval(img, O.quant_table(it.quality))
            spent += time.perf_counter() - t1
            blocks += (it.height // 8) * (it.width // 8)
            n += 1
        mean_all = self.nb / len(self.items)
        return {"value": blocks / spent / 1e6, "unit": "Mblocks/s", "cores": _oracle_threads(),
                "kind": "oracle",
                "sample": f"{n} of the 1000 planes in a seeded random order ({blocks} blocks, "
                          f"{blocks / max(n, 1):.0f} per plane against {mean_all:.0f} over the "
                          "batch), forward + exact quantisation + float64 inverse + SSE"}


class SingleImage:
    """One 512 x 512 plane (seed 0), r = 10: forward to int32 coefficients,
    retention, inverse to float32 pixels and the exact error sum in one launch,
    then the sum read back and its PSNR (the small configuration of Section 3's
    procedure).  Steps run back to back; `latency()` times single synchronous
    calls (launch to PSNR on the host)."""
    name = "single-512x512-r10"
    workload_key = "single"
    dtype = "int32+int64"

    def __init__(self, size=512, r=10):
        import torch
        from paper_1402_6034_amd import rdct as R, synth
        self.R = R
        self.size, self.r = size, r
        self.img = synth.render(0, size, size, device="cuda")
        self.nb = (size // 8) ** 2
        self.sel = R.select(R.SEL_ZIGZAG, r=r)
        self.coef = torch.empty((self.nb, 64), dtype=torch.int32, device="cuda")
        self.rec = torch.empty((size, size), dtype=torch.float32, device="cuda")
        self.sse = torch.empty(1, dtype=torch.int64, device="cuda")
        self.host = torch.empty(1, dtype=torch.int64, pin_memory=True)
        self.psnr = None

    def launch(self, i=0):
        self.R.compress_eval(self.img, self.sel, 1, self.R.COEF_I32, True, sse=self.sse,
                             coef=self.coef, recon_out=self.rec)

    kernel_launch = launch

    def step(self):
        self.launch()
        self.host.copy_(self.sse, non_blocking=True)
        import torch
        torch.cuda.current_stream().synchronize()
        self.psnr = self.R.rdct_psnr(int(self.host[0]), self.R.SEL_ZIGZAG, self.size, self.size)

    blocks_per_step = property(lambda self: self.nb)
    # 64 B of pixels in, 256 B of int32 coefficients and 256 B of float pixels out.
    bytes_per_block = 64 + 256 + 256

    def latency(self, reps=200):
        """Median and p99 microseconds of one synchronous call (launch, read-back, PSNR)."""
        import numpy as np
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            self.step()
            ts.append((time.perf_counter() - t0) * 1e6)
        return {"p50_us": round(float(np.percentile(ts, 50)), 2),
                "p99_us": round(float(np.percentile(ts, 99)), 2), "psnr_db": round(self.psnr, 4)}

    def config(self):
        return {"workload": self.name, "plane": [self.size, self.size], "blocks": self.nb,
                "r": self.r, "coef": "int32", "recon": "float32"}

    def report(self):
        return {"latency": self.latency()}

    def cpu_baseline(self, budget_s):
        import oracle as O
        img = self.img.cpu().numpy()
        t0 = time.perf_counter()
        n = 0
        while time.perf_counter() - t0 < budget_s:
            O.retention_eval(img, [self.r], recon_r=self.r)
            n += 1
        dt = time.perf_counter() - t0
        return {"value": n * self.nb / dt / 1e6, "unit": "Mblocks/s", "cores": _oracle_threads(),
                "kind": "oracle",
                "sample": f"{n} passes over the 512 x 512 plane (forward, r = 10, inverse, SSE)"}


# rdct_stream patterns: name, and the library kernel whose read:write mix it matches.
STREAM_PATTERNS = {0: ("read", None), 1: ("write", None), 2: ("copy", None),
                   3: ("r1w2", "frame quantiser, 64 B in / 128 B out per block"),
                   4: ("r1w6", "ragged batch, 64 B in / 384 B out per block")}


class StreamCalibration:
    """Practical HBM ceilings: the library's streaming calibration kernel in each
    read:write mix (pure read, pure write, 1:1, 1:2 as the frame quantiser, 1:6
    as the ragged batch), nontemporal or regular loads and stores, one unit per
    wave (as the frame kernel's chunks) or persistent workgroups (as the batch
    kernel).  The 1:2 mix runs at the frame's size (64 MiB read, 128 MiB written
    per launch, six buffer sets rotating past the 256 MB last-level cache); the
    others move 1 GiB or more per launch.  `value` is the best 1:2 rate."""
    name = "stream-calibration"
    workload_key = "stream"
    dtype = "u8"

    def __init__(self):
        import torch
        from paper_1402_6034_amd import rdct as R
        self.R = R
        self.units = {0: 131072, 1: 65536, 2: 65536, 3: 8192, 4: 208144}
        self.sets = {0: 1, 1: 1, 2: 1, 3: 6, 4: 1}
        self.bufs = {}
        for p, u in self.units.items():
            rb, wb = R.rdct_stream_unit_bytes(p)
            self.bufs[p] = [(torch.ones(max(u * rb, 16), dtype=torch.uint8, device="cuda"),
                             torch.empty(max(u * wb, 1024), dtype=torch.uint8, device="cuda"))
                            for _ in range(self.sets[p])]
        self.results = []
        self.best = {}
        self.no_sweep = False

    def run_case(self, p, flags, wpc, reps=20):
        import torch
        bufs, u = self.bufs[p], self.units[p]
        rb, wb = self.R.rdct_stream_unit_bytes(p)

        def one(i):
            src, dst = bufs[i % len(bufs)]
            self.R.rdct_stream(src if rb else None, dst, u, p, flags, wpc)
        rounds = sorted(event_time_ms(one, reps) for _ in range(3))
        ms = rounds[1]
        gbs = u * (rb + wb) / (ms * 1e-3) / 1e9
        return ms, gbs

    def sweep(self):
        for p in self.units:
            for flags in range(8):
                for wpc in (0, 2, 4, 8):
                    ms, gbs = self.run_case(p, flags, wpc)
                    row = {"pattern": STREAM_PATTERNS[p][0], "nt_loads": bool(flags & 1),
                           "nt_stores": bool(flags & 2), "xcd_ranges": bool(flags & 4),
                           "grid": "one unit per wave" if wpc == 0 else f"{wpc} WGs/CU persistent",
                           "ms": round(ms, 5), "GB/s": round(gbs, 1)}
                    self.results.append(row)
                    b = self.best.get(p)
                    if b is None or gbs > b["GB/s"]:
                        self.best[p] = row
                    log(f"[bench] stream {row}")

    def launch(self, i=0):
        """The 1:2 mix at the frame's size: regular loads, nontemporal stores, two
        persistent workgroups per CU (the fastest 1:2 form measured)."""
        src, dst = self.bufs[3][i % self.sets[3]]
        self.R.rdct_stream(src, dst, self.units[3], 3, 2, 2)

    kernel_launch = launch

    def step(self):
        if not self.results and not self.no_sweep:
            self.sweep()
        self.launch()

    blocks_per_step = property(lambda self: self.units[3] * 128)
    bytes_per_block = 64 + 128

    def config(self):
        return {"workload": self.name,
                "sizes": {STREAM_PATTERNS[p][0]: {"units": u, "bytes_per_unit":
                                                  list(self.R.rdct_stream_unit_bytes(p))}
                          for p, u in self.units.items()}}

    def report(self):
        return {"stream": {"best": {STREAM_PATTERNS[p][0]: dict(b, matches=STREAM_PATTERNS[p][1])
                                    for p, b in self.best.items()},
                           "all": self.results}}

    def cpu_baseline(self, budget_s):
        return None


def serving_leg(n_requests, rate_hz=2000.0, pool=3, budget=8 << 30):
    """Poisson trace of compression requests (Y + 4:2:0 Cb/Cr planes, resolutions
    256x256 .. 3840x2160, r uniform in 1..45) replayed in real time against the
    batching server and against the plain path (one synchronous launch per
    plane); p50/p99 latency from arrival to completion, throughput, and whether
    the two give identical error sums."""
    import numpy as np
    from paper_1402_6034_amd import rdct as R, serve as S, synth
    trace = synth.serve_trace(0, n_requests, rate_hz, pool=pool)
    planes = {}
    for q in trace:
        if q.seed not in planes:
            ch, cw = synth.chroma_shape(q.height, q.width)
            planes[q.seed] = [synth.render(q.seed, q.height, q.width, device="cuda").cpu().numpy(),
                              synth.render(q.seed + 1, ch, cw, device="cuda").cpu().numpy(),
                              synth.render(q.seed + 2, ch, cw, device="cuda").cpu().numpy()]
    sels = [R.select(R.SEL_ZIGZAG, r=q.r) for q in trace]
    idx = {id(q): i for i, q in enumerate(trace)}
    out = {"requests": n_requests, "rate_hz": rate_hz, "budget_bytes": budget,
           "mean_pixels_per_request": float(np.mean([sum(p.size for p in planes[q.seed]) for q in trace]))}
    results = {}
    blocks = sum(R.rdct_num_blocks(p.shape[1], p.shape[0]) for q in trace for p in planes[q.seed])
    for name, plain in (("batched", False), ("plain", True)):
        srv = S.Server(budget_bytes=budget, n_streams=2, plain=plain)
        # Warm-up (kernel loading, first launches): one request per pool entry.
        for k, key in enumerate(planes):
            srv.submit(planes[key], sels[0], tag=10 ** 9 + k)
        srv.drain(60000)
        while srv.poll(256):
            pass
        res = {}
        for mode, speed in (("trace", 1.0), ("burst", 1e9)):
            done, wall, busy = S.replay(srv, trace, lambda q: planes[q.seed],
                                        lambda q: sels[idx[id(q)]], timeout_s=300.0, speed=speed)
            lat = S.latency_stats(done)
            res[mode] = {"p50_ms": round(lat["p50_ms"], 4), "p99_ms": round(lat["p99_ms"], 4),
                         "mean_ms": round(lat["mean_ms"], 4), "max_ms": round(lat["max_ms"], 4),
                         "req_per_s": round(n_requests / wall, 1),
                         "mblocks_per_s": round(blocks / wall / 1e6, 2), "busy_retries": busy}
            if mode == "trace":
                results[name] = done
            log(f"[bench] serving {name} {mode}: p50 {lat['p50_ms']:.3f} ms, "
                f"p99 {lat['p99_ms']:.3f} ms, {n_requests / wall:.0f} req/s")
        st = srv.stats()
        srv.close()
        res["launches"] = st["batches"]
        res["peak_device_bytes"] = st["peak_device_bytes"]
        out[name] = res
    out["identical_sse"] = all(results["batched"][i]["sse"] == results["plain"][i]["sse"]
                               for i in range(n_requests))
    return out


WORKLOADS = {"frame": FrameQuant, "sweep": RetentionSweep, "ragged": RaggedBatch,
             "quality": QualitySweep, "codec": CodecFrame, "single": SingleImage,
             "stream": StreamCalibration, "inverse": InverseFrame}


def _pool_worker(job):
    """One worker of the multi-core oracle baseline: renders its planes on the
    CPU (not timed) and times the oracle on each until its budget is spent."""
    budget_s, items = job
    from threadpoolctl import threadpool_limits
    import oracle as O
    from paper_1402_6034_amd import synth
    blocks, spent = 0, 0.0
    with threadpool_limits(limits=1):
        for it in items:
            img = synth.render_np(it.seed, it.height, it.width)
            t0 = time.perf_counter()
            O.quant_eval(img, O.quant_table(it.quality))
            spent += time.perf_counter() - t0
            blocks += (it.height // 8) * (it.width // 8)
            if spent > budget_s:
                break
    return blocks, spent


def cpu_pool_baseline(budget_s):
    """The oracle on the ragged batch's planes over a pool of processes, one per
    core available to this process (at most 16), each single-threaded.  Runs
    before the GPU is initialised (the workers are forked).  Value: the sum of
    the workers' own rates (rendering excluded)."""
    import multiprocessing as mp
    from paper_1402_6034_amd import synth
    cores = min(16, len(os.sched_getaffinity(0)))
    items = sorted(synth.ragged_batch(0, 1000), key=lambda it: it.height * it.width)
    jobs = [(budget_s, items[k::cores]) for k in range(cores)]
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_pool_worker, jobs)
    rate = sum(b / t for b, t in res if t > 0) / 1e6
    blocks = sum(b for b, _ in res)
    return {"value": rate, "unit": "Mblocks/s", "cores": cores, "kind": "oracle",
            "sample": f"{cores} single-threaded processes, each on every {cores}-th of the 1000 "
                      f"planes in size order for ~{budget_s:g} s of oracle time ({blocks} blocks "
                      "in all; planes rendered on the CPU, same generator and sizes); forward + "
                      "exact quantisation + float64 inverse + SSE"}


def _oracle_threads():
    """The oracle runs in one process with its BLAS pool limited to one thread
    (see main), so it uses one core."""
    return 1


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="ragged", choices=sorted(WORKLOADS))
    ap.add_argument("--no-plain", action="store_true", help="skip the one-launch-per-plane comparison")
    ap.add_argument("--tuning-table", action="store_true",
                    help="ragged: time every geometry of the autotuner with and without graph "
                         "replay and add the table to the line")
    ap.add_argument("--no-sweep", action="store_true",
                    help="stream: time only the 1:2 kernel (no sweep of every variant)")
    ap.add_argument("--no-extras", action="store_true",
                    help="ragged: skip the frame and single-plane figures added to the line")
    ap.add_argument("--no-autotune", action="store_true",
                    help="ragged, sweep: use the tuning cache (or defaults) instead of tuning first")
    ap.add_argument("--geometry", default=None, metavar="WPGxWPC:XCD:STRIP",
                    help="ragged, sweep: run the strided layout at this geometry (e.g. 1x4:1:2) "
                         "instead of tuning (profiles of one geometry)")
    ap.add_argument("--serve-requests", type=int, default=None,
                    help="requests in the served trace (2000 req/s; 0 = skip the serving leg; "
                         "default 4000 with the ragged workload, else 0)")
    ap.add_argument("--planes-cache", default=None,
                    help="ragged, sweep, quality: .npy file holding the rendered planes (written if absent)")
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle time for the CPU baseline (0 = skip)")
    ap.add_argument("--cpu-pool-budget", type=float, default=4.0,
                    help="ragged: seconds of oracle time per process for the multi-core "
                         "baseline (0 = skip)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the run, copy MIB mebibytes device-to-device 3 times "
                         "(reference kernel for the FETCH_SIZE/WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.steps < 1 or args.warmup < 0:
        ap.error("--steps must be at least 1 and --warmup at least 0")
    if args.serve_requests is None:
        args.serve_requests = 4000 if args.workload == "ragged" else 0
    if args.gpus != 1:
        print("bench.py: measures one MI355X only; runs on several GPUs are not provided "
              "(planes and requests would shard across GPUs with no exchange but the per-plane "
              "error sums).", file=sys.stderr)
        sys.exit(2)

    cpu_pool = None
    if args.workload == "ragged" and args.cpu_budget > 0 and args.cpu_pool_budget > 0:
        log("[bench] timing the CPU oracle over a process pool (before GPU start-up)")
        cpu_pool = cpu_pool_baseline(args.cpu_pool_budget)
        log(f"[bench] pool oracle: {cpu_pool['value']:.3f} Mblocks/s on {cpu_pool['cores']} cores")

    import torch
    from paper_1402_6034_amd import rdct as R
    R.lib()
    torch.cuda.init()
    tune = not args.no_autotune and args.geometry is None
    if args.workload == "ragged":
        wl = RaggedBatch(planes_cache=args.planes_cache, autotune=tune)
    elif args.workload == "sweep":
        wl = RetentionSweep(autotune=tune, planes_cache=args.planes_cache)
    elif args.workload == "quality":
        wl = QualitySweep(planes_cache=args.planes_cache)
    else:
        wl = WORKLOADS[args.workload]()
    if args.geometry is not None and args.workload in ("ragged", "sweep"):
        size, xcd, strip = args.geometry.split(":")
        wpg, wpc = (int(v) for v in size.split("x"))
        wl.plan.set_tuning(R.Tuning(wpg, wpc, 0, R.LAYOUT_STRIDED, int(xcd), int(strip)))
        log(f"[bench] geometry set: strided, {wpg} waves/WG x {wpc} WGs/CU, XCD ranges {xcd}, "
            f"strip {strip}")
    if args.workload == "stream":
        wl.no_sweep = args.no_sweep

    for _ in range(args.warmup):
        wl.step()
    torch.cuda.synchronize()
    log(f"[bench] warmup done ({args.warmup} steps)")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if hasattr(wl, "submit"):
        # Two steps in flight: step k + 1 is enqueued before step k's sums are
        # read back and turned into PSNR, so host work overlaps the next kernel.
        for k in range(args.steps):
            wl.submit(k & 1)
            if k:
                wl.finish((k - 1) & 1)
        wl.finish((args.steps - 1) & 1)
    else:
        for _ in range(args.steps):
            wl.step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt * 1e3 / args.steps
    log(f"[bench] timed {args.steps} steps: {ms:.4f} ms/step")

    # Dominant kernel: average launch duration from HIP events.
    reps = max(20, args.steps)
    k_ms = event_time_ms(lambda i: wl.kernel_launch(i), reps)
    tr = traffic_record(wl.workload_key, geometry_tag(wl.config()))
    if getattr(wl, "roofline_kind", "hbm") == "alu":
        flops = wl.flops_per_launch
        achieved = flops / (k_ms * 1e-3) / 1e12
        roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                    "traffic": tr["bytes"] if tr else None,
                    "kernel_ms": round(k_ms, 5), "flops_per_launch": flops,
                    "kernel_source_sha256": kernel_source_hash(wl.workload_key)}
    else:
        nb = wl.blocks_per_step
        alg_bytes = int(round(nb * wl.bytes_per_block))
        achieved = alg_bytes / (k_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": tr["bytes"] if tr else None,
                    "kernel_ms": round(k_ms, 5), "bytes_per_launch": alg_bytes,
                    "kernel_source_sha256": kernel_source_hash(wl.workload_key)}
    if tr:
        roofline["traffic_read"] = tr["read"]
        roofline["traffic_write"] = tr["write"]
        if "profiler_us" in tr and "bytes_per_launch" in roofline:
            # The dominant kernel alone as rocprofv3 timed it in the committed
            # profile (the HIP-event figure above times a whole plan run, which
            # for the strided batch layout includes the small clearing launch).
            p_ms = tr["profiler_us"] * 1e-3
            roofline["profiler_kernel_ms"] = round(p_ms, 5)
            roofline["profiler_frac"] = round(
                roofline["bytes_per_launch"] / (p_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    valu = valu_record(wl.workload_key)
    if valu:
        # Issue rate of vector instructions against the chip's: every CU issues at
        # most one wave instruction per clock (4 SIMDs, a wave64 instruction each
        # 4 clocks).
        rate = valu / (k_ms * 1e-3) / 1e9
        peak = N_CU * CLOCK_GHZ
        roofline["valu_issue"] = {"achieved": round(rate, 1), "peak": round(peak, 1),
                                  "unit": "G wave-instructions/s", "frac": round(rate / peak, 4),
                                  "instructions_per_launch": valu}

    extras = {}
    if args.workload == "ragged" and args.tuning_table:
        log("[bench] tuning table")
        extras["tuning_table"] = wl.tuning_table()
    if args.workload == "ragged" and not args.no_extras:
        # The other configurations' headline figures beside the default line:
        # the 8192^2 quantisation frame (its kernel against the HBM peak) and one
        # 512^2 plane at r = 10 (throughput and single-call latency).
        fr = FrameQuant()
        f_ms = event_time_ms(lambda i: fr.kernel_launch(i), 60)
        f_bytes = fr.blocks_per_step * fr.bytes_per_block
        extras["frame"] = {"workload": fr.name, "kernel_ms": round(f_ms, 5),
                           "achieved_GBs": round(f_bytes / (f_ms * 1e-3) / 1e9, 2),
                           "frac": round(f_bytes / (f_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                           "bytes_per_launch": f_bytes,
                           "mblocks_per_s": round(fr.blocks_per_step / (f_ms * 1e-3) / 1e6, 1)}
        del fr
        one = SingleImage()
        for _ in range(20):
            one.step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(500):
            one.launch()
        torch.cuda.synchronize()
        s_ms = (time.perf_counter() - t1) * 1e3 / 500
        extras["single"] = {"workload": one.name, "us_per_image": round(s_ms * 1e3, 2),
                            "mblocks_per_s": round(one.nb / (s_ms * 1e-3) / 1e6, 1),
                            "synchronous_call": one.latency()}
        del one
        log(f"[bench] frame kernel {extras['frame']['kernel_ms']} ms "
            f"({extras['frame']['frac']} of peak); single 512^2 {extras['single']['us_per_image']} us")

    cpu = None
    if args.cpu_budget > 0:
        log("[bench] timing the CPU oracle on a sample")
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            cpu = wl.cpu_baseline(args.cpu_budget)

    value = wl.blocks_per_step / (ms * 1e-3) / 1e6
    unit = "Mblocks/s"
    if args.workload == "stream":
        # The calibration moves bytes, not blocks: its value is the 1:2 kernel's rate.
        value, unit = roofline["achieved"], "GB/s"
    plain = None
    if hasattr(wl, "plain") and not args.no_plain:
        log("[bench] timing the plain one-launch-per-plane path")
        plain = wl.plain()

    serving = None
    if args.serve_requests > 0:
        log("[bench] serving leg")
        serving = serving_leg(args.serve_requests)

    out = {"metric": METRIC, "value": round(value, 3), "unit": unit, "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": wl.dtype, "data": "synthetic", "config": wl.config(),
           "roofline": roofline, "cpu_baseline": cpu}
    if cpu_pool is not None:
        out["cpu_baseline_pool"] = cpu_pool
    if plain is not None:
        out["plain"] = plain
    if hasattr(wl, "report") and wl.report():
        out.update(wl.report())
    out.update(extras)
    if serving is not None:
        out["serving"] = serving
    print(json.dumps(out), flush=True)
    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {n} bytes x3 done")


if __name__ == "__main__":
    main()
