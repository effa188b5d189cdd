"""Python driver of the compression server (rdct_server_* in librdct).

`Server` wraps the C-ABI one for one (argument marshalling only); `replay`
plays an open-loop arrival trace against a server -- one thread submits each
request at its arrival time, the caller's thread collects completions -- and
returns per-request latencies.
"""
from __future__ import annotations

import ctypes
import gc
import threading
import time
from ctypes import POINTER, c_double, c_int32, c_int64, c_uint8, c_uint64, c_void_p

import numpy as np

from . import rdct as R


class ServerCfg(ctypes.Structure):
    _fields_ = [("budget_bytes", c_int64), ("staging_bytes", c_int64), ("max_inflight", c_int32),
                ("max_batch_planes", c_int32), ("n_streams", c_int32), ("plain", c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("planes", POINTER(c_uint8) * 3), ("width", c_int32 * 3), ("height", c_int32 * 3),
                ("pitch", c_int64 * 3), ("n_planes", c_int32), ("sel", R.Select),
                ("user_tag", c_uint64)]


class Completion(ctypes.Structure):
    _fields_ = [("ticket", c_uint64), ("user_tag", c_uint64), ("status", c_int32),
                ("n_planes", c_int32), ("sse", c_uint64 * 3), ("psnr", c_double * 3),
                ("t_submit_us", c_double), ("t_launch_us", c_double), ("t_done_us", c_double),
                ("batch_planes", c_int32), ("reserved", c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("submitted", c_int64), ("completed", c_int64), ("cancelled", c_int64),
                ("rejected", c_int64), ("batches", c_int64), ("planes", c_int64),
                ("blocks", c_int64), ("peak_device_bytes", c_int64),
                ("device_bytes_in_use", c_int64), ("pending", c_int32), ("inflight", c_int32)]


def declare(L):
    P = c_void_p
    L.rdct_server_create.argtypes = [POINTER(ServerCfg), POINTER(c_void_p)]
    L.rdct_server_submit.argtypes = [P, POINTER(Request), POINTER(c_uint64)]
    L.rdct_server_poll.argtypes = [P, POINTER(Completion), c_int32, POINTER(c_int32), c_int32]
    L.rdct_server_cancel.argtypes = [P, c_uint64]
    L.rdct_server_drain.argtypes = [P, c_int32]
    L.rdct_server_stats.argtypes = [P, POINTER(Stats)]
    L.rdct_server_destroy.argtypes = [P]
    for f in ("rdct_server_create", "rdct_server_submit", "rdct_server_poll", "rdct_server_cancel",
              "rdct_server_drain", "rdct_server_stats"):
        getattr(L, f).restype = c_int32
    L.rdct_server_destroy.restype = None


class Server:
    def __init__(self, budget_bytes=8 << 30, staging_bytes=0, max_inflight=0, max_batch_planes=0,
                 n_streams=0, plain=False):
        L = R.lib()
        self.cfg = ServerCfg(budget_bytes, staging_bytes, max_inflight, max_batch_planes, n_streams,
                             1 if plain else 0)
        h = c_void_p()
        R._check(L.rdct_server_create(ctypes.byref(self.cfg), ctypes.byref(h)), "rdct_server_create")
        self.h = h
        self._buf = (Completion * 256)()

    def submit(self, planes, sel, tag=0):
        """planes: list of 1..3 C-contiguous uint8 numpy arrays (host)."""
        req = Request()
        req.n_planes = len(planes)
        for i, p in enumerate(planes):
            req.planes[i] = p.ctypes.data_as(POINTER(c_uint8))
            req.height[i], req.width[i] = p.shape
            req.pitch[i] = p.strides[0]
        req.sel = sel
        req.user_tag = tag
        t = c_uint64()
        st = R.lib().rdct_server_submit(self.h, ctypes.byref(req), ctypes.byref(t))
        if st != R.OK:
            raise R.RdctError(st, "rdct_server_submit")
        return t.value

    def try_submit(self, planes, sel, tag=0):
        """Like submit but returns the status instead of raising (ticket or None)."""
        try:
            return R.OK, self.submit(planes, sel, tag)
        except R.RdctError as e:
            return e.status, None

    def poll(self, max_n=256, wait_us=0):
        n = c_int32()
        R._check(R.lib().rdct_server_poll(self.h, self._buf, min(max_n, 256), ctypes.byref(n),
                                          wait_us), "rdct_server_poll")
        out = []
        for c in self._buf[:n.value]:
            out.append({"ticket": c.ticket, "tag": c.user_tag, "status": c.status,
                        "sse": list(c.sse[:c.n_planes]), "psnr": list(c.psnr[:c.n_planes]),
                        "t_submit_us": c.t_submit_us, "t_launch_us": c.t_launch_us,
                        "t_done_us": c.t_done_us, "batch_planes": c.batch_planes})
        return out

    def cancel(self, ticket):
        return R.lib().rdct_server_cancel(self.h, ticket)

    def drain(self, timeout_ms=60000):
        return R.lib().rdct_server_drain(self.h, timeout_ms)

    def stats(self):
        s = Stats()
        R._check(R.lib().rdct_server_stats(self.h, ctypes.byref(s)), "rdct_server_stats")
        return {f: getattr(s, f) for f, _ in Stats._fields_}

    def close(self):
        if self.h:
            R.lib().rdct_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def replay(server, trace, planes_of, sel_of, timeout_s=120.0, speed=1.0):
    """Submit trace[i] at its arrival time (scaled by 1/speed) and collect every
    completion.  planes_of(req) -> list of host planes; sel_of(req) -> Select.
    Returns (completions by tag, wall seconds, number of BUSY retries)."""
    done = {}
    busy = [0]
    err = []
    t_start = 0.0

    def submitter():
        try:
            for i, req in enumerate(trace):
                target = t_start + req.arrival_s / speed
                while True:
                    now = time.perf_counter()
                    if now >= target:
                        break
                    time.sleep(min(target - now, 0.0005))
                planes = planes_of(req)
                sel = sel_of(req)
                while True:
                    st, _ = server.try_submit(planes, sel, tag=i)
                    if st == R.OK:
                        break
                    if st != R.ERR_BUSY:
                        raise R.RdctError(st, "submit")
                    busy[0] += 1
                    time.sleep(0.0002)
        except Exception as e:  # pragma: no cover
            err.append(e)

    # The cyclic garbage collector is paused for the replay: its pauses (tens of
    # milliseconds with many live objects) would otherwise show up as request
    # latency on whichever requests are in flight.
    gc.collect()
    gc_was_enabled = gc.isenabled()
    gc.disable()
    t_start = time.perf_counter()
    th = threading.Thread(target=submitter, daemon=True)
    th.start()
    try:
        deadline = time.perf_counter() + timeout_s
        while len(done) < len(trace):
            for c in server.poll(256, wait_us=2000):
                # Latency from the request's arrival time to its collection here.
                c["latency_ms"] = (time.perf_counter() - t_start
                                   - trace[c["tag"]].arrival_s / speed) * 1e3
                done[c["tag"]] = c
            if err:
                raise err[0]
            if time.perf_counter() > deadline:
                raise TimeoutError(f"replay: {len(done)} of {len(trace)} completed")
        th.join()
    finally:
        if gc_was_enabled:
            gc.enable()
    return done, time.perf_counter() - t_start, busy[0]


def latency_stats(done):
    lat = np.array([c["latency_ms"] for c in done.values()])
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max())}
