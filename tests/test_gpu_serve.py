"""Compression server: continuous batching gives each request the result it gets
alone (bit-exact error sums), the budget is enforced, and queueing, cancellation
and rejection behave."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1402_6034_amd import synth

pytestmark = pytest.mark.gpu

R = pytest.importorskip("paper_1402_6034_amd.rdct")
S = pytest.importorskip("paper_1402_6034_amd.serve")


def request_planes(h, w, seed):
    y = synth.render_np(seed, h, w)
    ch, cw = synth.chroma_shape(h, w)
    return [y, synth.render_np(seed + 1, ch, cw), synth.render_np(seed + 2, ch, cw)]


def alone(planes, sel):
    out = []
    for p in planes:
        s, _, _ = R.compress_eval(torch.from_numpy(p).cuda(), sel, 1)
        torch.cuda.synchronize()
        out.append(int(s.cpu()[0]))
    return out


def small_trace(n, seed):
    rng = np.random.default_rng(seed)
    res = [(64, 64), (120, 160), (72, 128), (135, 240), (270, 480)]
    reqs = []
    for i in range(n):
        h, w = res[int(rng.integers(0, len(res)))]
        reqs.append((request_planes(h, w, 1000 * seed + 3 * i), int(rng.integers(1, 46))))
    return reqs


@pytest.mark.parametrize("plain", [False, True])
def test_results_identical_alone_and_in_mix(plain):
    reqs = small_trace(24, 1)
    srv = S.Server(budget_bytes=256 << 20, n_streams=2, plain=plain)
    tickets = {}
    for i, (planes, r) in enumerate(reqs):
        tickets[srv.submit(planes, R.select(R.SEL_ZIGZAG, r=r), tag=i)] = i
    assert srv.drain(60000) == R.OK
    got = {}
    while len(got) < len(reqs):
        for c in srv.poll(256, wait_us=1000):
            got[c["tag"]] = c
    for i, (planes, r) in enumerate(reqs):
        c = got[i]
        assert c["status"] == R.OK
        assert c["sse"] == alone(planes, R.select(R.SEL_ZIGZAG, r=r)), i
        for k, p in enumerate(planes):
            h, w = p.shape
            assert c["psnr"][k] == R.rdct_psnr(c["sse"][k], R.SEL_ZIGZAG, w, h)
    # Oracle on one request.
    ref = O.retention_eval(reqs[3][0][1], [reqs[3][1]])
    assert got[3]["sse"][1] == ref["sse_num"][reqs[3][1]]
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["device_bytes_in_use"] <= 256
    srv.close()


def test_tiny_budget_forces_queueing_and_is_never_exceeded():
    reqs = small_trace(12, 2)
    reqs += [(request_planes(540, 960, 999), 7)] * 2
    # Room for about two of the largest requests at a time.
    largest = max(sum(p.size for p in planes) for planes, _ in reqs)
    budget = max(1 << 20, int(2.5 * largest) + (64 << 10))
    srv = S.Server(budget_bytes=budget, staging_bytes=64 << 20, n_streams=2)
    for i, (planes, r) in enumerate(reqs):
        srv.submit(planes, R.select(R.SEL_ZIGZAG, r=r), tag=i)
    assert srv.drain(60000) == R.OK
    got = {}
    while len(got) < len(reqs):
        for c in srv.poll(256, wait_us=1000):
            got[c["tag"]] = c
    for i, (planes, r) in enumerate(reqs):
        assert got[i]["sse"] == alone(planes, R.select(R.SEL_ZIGZAG, r=r))
    st = srv.stats()
    assert st["peak_device_bytes"] <= budget
    assert st["batches"] >= 2
    srv.close()


def test_oversize_request_is_rejected_without_blocking():
    srv = S.Server(budget_bytes=1 << 20)
    big = [np.zeros((2048, 2048), dtype=np.uint8)]
    st, t = srv.try_submit(big, R.select(R.SEL_ZIGZAG, r=10))
    assert st == R.ERR_BUDGET and t is None
    ok = [np.full((64, 64), 9, dtype=np.uint8)]
    st, t = srv.try_submit(ok, R.select(R.SEL_ZIGZAG, r=10))
    assert st == R.OK
    assert srv.drain(10000) == R.OK
    srv.close()


def test_invalid_request_is_rejected():
    srv = S.Server(budget_bytes=16 << 20)
    st, _ = srv.try_submit([np.zeros((8, 8), np.uint8)], R.select(R.SEL_ZIGZAG, r=0))
    assert st == R.ERR_INVALID_ARG
    assert srv.cancel(12345) == R.ERR_NOT_FOUND
    srv.close()


def test_cancel_pending_request():
    # max_inflight = 1 and one stream: later requests wait in the queue.
    srv = S.Server(budget_bytes=64 << 20, n_streams=1, max_inflight=1)
    reqs = small_trace(6, 3)
    tickets = [srv.submit(p, R.select(R.SEL_ZIGZAG, r=r), tag=i) for i, (p, r) in enumerate(reqs)]
    st = srv.cancel(tickets[-1])
    assert st in (R.OK, R.ERR_BUSY)
    assert srv.drain(60000) == R.OK
    got = {}
    while len(got) < len(reqs):
        for c in srv.poll(256, wait_us=1000):
            got[c["tag"]] = c
    if st == R.OK:
        assert got[5]["status"] == R.ERR_CANCELLED
    for i in range(5):
        assert got[i]["status"] == R.OK
    srv.close()


def test_quant_requests():
    planes = request_planes(96, 160, 77)
    sel = R.select(R.SEL_QUANT, quality=37, level_shift=128)
    srv = S.Server(budget_bytes=64 << 20)
    srv.submit(planes, sel, tag=0)
    assert srv.drain(20000) == R.OK
    c = srv.poll(4, wait_us=1000)[0]
    assert c["sse"] == alone(planes, sel)
    ref = O.quant_eval(planes[0], O.quant_table(37))
    assert abs(c["psnr"][0] - ref["psnr"]) <= 1e-3
    srv.close()


def test_replay_trace():
    reqs = small_trace(40, 4)
    trace = [synth.ServeRequest(arrival_s=0.0005 * i, height=p[0].shape[0], width=p[0].shape[1],
                                r=r, seed=i) for i, (p, r) in enumerate(reqs)]
    srv = S.Server(budget_bytes=256 << 20)
    done, wall, busy = S.replay(srv, trace, lambda q: reqs[q.seed][0],
                                lambda q: R.select(R.SEL_ZIGZAG, r=q.r))
    assert len(done) == 40
    for i, (p, r) in enumerate(reqs[:5]):
        assert done[i]["sse"] == alone(p, R.select(R.SEL_ZIGZAG, r=r))
    lat = S.latency_stats(done)
    assert 0 < lat["p50_ms"] <= lat["p99_ms"]
    srv.close()


def test_quant_requests_in_mix_equal_alone():
    # Whole-block planes (scored in the coefficient domain) and planes with
    # partial blocks (odd 4:2:0 chroma sizes, scored pixel by pixel) share
    # batches; each plane's sum has the bits it has alone.
    reqs = small_trace(30, 5)
    rng = np.random.default_rng(5)
    sels = [R.select(R.SEL_QUANT, quality=int(q), level_shift=128)
            for q in rng.integers(10, 91, len(reqs))]
    shapes = [p.shape for planes, _ in reqs for p in planes]
    assert any(h % 8 or w % 8 for h, w in shapes) and any(h % 8 == 0 and w % 8 == 0 for h, w in shapes)
    srv = S.Server(budget_bytes=256 << 20, n_streams=2)
    for i, ((planes, _), sel) in enumerate(zip(reqs, sels)):
        srv.submit(planes, sel, tag=i)
    assert srv.drain(60000) == R.OK
    got = {}
    while len(got) < len(reqs):
        for c in srv.poll(256, wait_us=1000):
            got[c["tag"]] = c
    for i, ((planes, _), sel) in enumerate(zip(reqs, sels)):
        assert got[i]["status"] == R.OK
        assert got[i]["sse"] == alone(planes, sel), i
    assert srv.stats()["batches"] < len(reqs)
    srv.close()


def test_metadata_bound_batches_with_a_small_budget():
    # A 1 MiB budget: each stream's metadata region holds far fewer requests
    # than are queued, so batches are cut by metadata, and every request still
    # completes with its own result.
    srv = S.Server(budget_bytes=1 << 20, staging_bytes=4 << 20, n_streams=2)
    planes = [synth.render_np(7, 64, 64), synth.render_np(8, 32, 32), synth.render_np(9, 32, 32)]
    sels = [R.select(R.SEL_QUANT, quality=q, level_shift=128) for q in range(10, 90)]
    for i, sel in enumerate(sels):
        srv.submit(planes, sel, tag=i)
    assert srv.drain(60000) == R.OK
    got = {}
    while len(got) < len(sels):
        for c in srv.poll(256, wait_us=1000):
            got[c["tag"]] = c
    for i in (0, 17, 79):
        assert got[i]["sse"] == alone(planes, sels[i])
    st = srv.stats()
    assert st["completed"] == len(sels) and st["batches"] >= 2
    srv.close()
