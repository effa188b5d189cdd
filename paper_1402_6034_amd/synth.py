"""Seeded synthetic 8-bit greyscale planes and workload descriptions.

The paper evaluates on 45 public 512x512 8-bit greyscale photographs (Section 3).
Those images are not available here, so every workload is built from a seeded
synthetic field with the same shape, size and bit depth: a smooth background made
of anisotropic Gaussian bumps, a few step edges and pixel noise.

This module holds none of the transform's arithmetic.  It only produces input
planes and workload descriptions; the CPU oracle tests and the GPU path consume
the very same arrays it returns.

Field (normalised coordinates u, v in [0, 1), pixel centres at (x + 1/2) / W):
  draws from numpy PCG64(seed), in this order:
    base b ~ U(64, 192)
    16 bumps: amplitude ~ U(-80, 80), centre ~ U(0,1)^2,
              sigma_u, sigma_v ~ logU(0.02, 0.25), angle ~ U(0, pi)
    4 step edges: point ~ U(0,1)^2, normal angle ~ U(0, 2 pi), height ~ U(-40, 40)
  then i.i.d. N(0, 2^2) noise per pixel from a torch generator seeded with `seed`
  on the rendering device, and uint8 = clip(floor(field + 1/2), 0, 255).
Rendering the same seed at 16x the resolution gives the same picture at 16x scale.
The noise stream depends on the device that renders the plane (CPU and GPU torch
generators differ); every check feeds one rendered array to both sides.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

N_BUMPS = 16
N_EDGES = 4
NOISE_SIGMA = 2.0


@dataclass(frozen=True)
class FieldParams:
    base: float
    bumps: np.ndarray  # (N_BUMPS, 6): amp, cu, cv, sigma_u, sigma_v, angle
    edges: np.ndarray  # (N_EDGES, 4): pu, pv, normal angle, height
    seed: int


def field_params(seed: int) -> FieldParams:
    rng = np.random.Generator(np.random.PCG64(seed))
    base = rng.uniform(64.0, 192.0)
    bumps = np.empty((N_BUMPS, 6))
    for j in range(N_BUMPS):
        amp = rng.uniform(-80.0, 80.0)
        cu, cv = rng.uniform(0.0, 1.0, size=2)
        su, sv = np.exp(rng.uniform(math.log(0.02), math.log(0.25), size=2))
        ang = rng.uniform(0.0, math.pi)
        bumps[j] = (amp, cu, cv, su, sv, ang)
    edges = np.empty((N_EDGES, 4))
    for j in range(N_EDGES):
        pu, pv = rng.uniform(0.0, 1.0, size=2)
        phi = rng.uniform(0.0, 2.0 * math.pi)
        h = rng.uniform(-40.0, 40.0)
        edges[j] = (pu, pv, phi, h)
    return FieldParams(base=base, bumps=bumps, edges=edges, seed=seed)


def render(seed: int, height: int, width: int, device="cpu", noise: bool = True,
           row_chunk: int = 2048) -> torch.Tensor:
    """Render the seeded field as a (height, width) uint8 tensor on `device`."""
    p = field_params(seed)
    dev = torch.device(device)
    out = torch.empty((height, width), dtype=torch.uint8, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed) & 0x7FFFFFFFFFFFFFFF)
    u = (torch.arange(width, device=dev, dtype=torch.float64) + 0.5) / width
    for y0 in range(0, height, row_chunk):
        y1 = min(height, y0 + row_chunk)
        v = (torch.arange(y0, y1, device=dev, dtype=torch.float64) + 0.5) / height
        uu = u[None, :]
        vv = v[:, None]
        f = torch.full((y1 - y0, width), p.base, dtype=torch.float64, device=dev)
        for amp, cu, cv, su, sv, ang in p.bumps:
            du = uu - cu
            dv = vv - cv
            ca, sa = math.cos(ang), math.sin(ang)
            a = du * ca + dv * sa
            b = dv * ca - du * sa
            f += amp * torch.exp(-(a * a) / (2.0 * su * su) - (b * b) / (2.0 * sv * sv))
        for pu, pv, phi, h in p.edges:
            side = (uu - pu) * math.cos(phi) + (vv - pv) * math.sin(phi)
            f += torch.where(side > 0, h, 0.0)
        if noise:
            f += NOISE_SIGMA * torch.randn((y1 - y0, width), generator=gen,
                                           dtype=torch.float64, device=dev)
        out[y0:y1] = torch.clamp(torch.floor(f + 0.5), 0.0, 255.0).to(torch.uint8)
    return out


def render_np(seed: int, height: int, width: int, noise: bool = True) -> np.ndarray:
    """CPU rendering as a numpy uint8 array."""
    return render(seed, height, width, device="cpu", noise=noise).numpy()


# ---------------------------------------------------------------------------
# Workload descriptions (sizes, qualities, retention counts, arrival traces)
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class RaggedItem:
    height: int
    width: int
    quality: int
    seed: int


def ragged_batch(seed: int = 0, n: int = 1000, lo: int = 64, hi: int = 4096,
                 q_lo: int = 10, q_hi: int = 90) -> list[RaggedItem]:
    """Ragged batch: width and height independently log-uniform in [lo, hi],
    rounded to multiples of 8; quality uniform in q_lo..q_hi; image i is rendered
    from seed 1_000_000 * (seed + 1) + i."""
    rng = np.random.Generator(np.random.PCG64(seed))
    items = []
    for i in range(n):
        w = int(8 * round(math.exp(rng.uniform(math.log(lo), math.log(hi))) / 8.0))
        h = int(8 * round(math.exp(rng.uniform(math.log(lo), math.log(hi))) / 8.0))
        q = int(rng.integers(q_lo, q_hi + 1))
        items.append(RaggedItem(height=h, width=w, quality=q,
                                seed=1_000_000 * (seed + 1) + i))
    return items


SERVE_RESOLUTIONS = ((256, 256), (480, 640), (720, 1280), (1080, 1920), (2160, 3840))
SERVE_PROBS = (0.3, 0.3, 0.2, 0.15, 0.05)


@dataclass(frozen=True)
class ServeRequest:
    arrival_s: float
    height: int   # luma plane; chroma planes are ceil(h/2) x ceil(w/2) (4:2:0)
    width: int
    r: int
    seed: int     # luma seed; Cb and Cr use seed + 1 and seed + 2


def serve_trace(seed: int = 0, n: int = 2000, rate_hz: float = 2000.0,
                r_lo: int = 1, r_hi: int = 45, pool: int = 0) -> list[ServeRequest]:
    """Open-loop Poisson trace: exponential gaps of mean 1/rate_hz, resolution from
    SERVE_RESOLUTIONS with SERVE_PROBS, r uniform in r_lo..r_hi.  With pool > 0
    the image seeds cycle through `pool` images per resolution (to bound the
    host memory spent on rendered planes)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate_hz)
        ri = int(rng.choice(len(SERVE_RESOLUTIONS), p=SERVE_PROBS))
        r = int(rng.integers(r_lo, r_hi + 1))
        h, w = SERVE_RESOLUTIONS[ri]
        k = (i % pool) if pool > 0 else i
        out.append(ServeRequest(arrival_s=t, height=h, width=w, r=r,
                                seed=10_000_000 * (seed + 1) + 3 * (ri * 100_000 + k)))
    return out


def chroma_shape(height: int, width: int) -> tuple[int, int]:
    """4:2:0 chroma plane size for a luma plane of the given size."""
    return (height + 1) // 2, (width + 1) // 2
