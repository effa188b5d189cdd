"""Input generator checks (CPU): determinism, ranges, workload descriptions."""
import numpy as np

from paper_1402_6034_amd import synth


def test_render_deterministic_and_in_range():
    a = synth.render_np(3, 40, 56)
    b = synth.render_np(3, 40, 56)
    c = synth.render_np(4, 40, 56)
    assert a.dtype == np.uint8 and a.shape == (40, 56)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)
    assert 0 < a.std() < 120


def test_same_picture_at_higher_resolution():
    # Noise-free renderings at 1x and 4x agree after 4x4 averaging (smooth field).
    lo = synth.render_np(7, 64, 64, noise=False).astype(float)
    hi = synth.render_np(7, 256, 256, noise=False).astype(float)
    down = hi.reshape(64, 4, 64, 4).mean(axis=(1, 3))
    assert np.median(np.abs(down - lo)) < 2.0


def test_ragged_batch_description():
    items = synth.ragged_batch(0, 1000)
    assert len(items) == 1000
    ws = np.array([i.width for i in items])
    hs = np.array([i.height for i in items])
    qs = np.array([i.quality for i in items])
    assert np.all(ws % 8 == 0) and np.all(hs % 8 == 0)
    assert ws.min() >= 64 and ws.max() <= 4096 and hs.min() >= 64 and hs.max() <= 4096
    assert qs.min() >= 10 and qs.max() <= 90
    assert synth.ragged_batch(0, 10) == items[:10]
    px = float(np.sum(ws.astype(np.int64) * hs))
    assert 0.6e9 < px < 1.3e9   # log-uniform sides: E[w h] ~ 0.94 G pixels for 1000 images


def test_serve_trace():
    tr = synth.serve_trace(0, 4000)
    gaps = np.diff([0.0] + [r.arrival_s for r in tr])
    assert abs(gaps.mean() - 0.5e-3) < 0.05e-3
    assert all(1 <= r.r <= 45 for r in tr)
    res = [(r.height, r.width) for r in tr]
    frac = res.count((256, 256)) / len(res)
    assert 0.25 < frac < 0.35
    assert synth.chroma_shape(1080, 1920) == (540, 960)
