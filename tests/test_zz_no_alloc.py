"""The allocation-free metric entry point (jet_km1_static) against jet_km1, through the C ABI.

jet_km1_static keeps its per-workgroup partial sums in a static device array shared by every call
on the GPU.  Two calls in a row, the second on a smaller hypergraph (fewer slots used, stale slots
of the first call left behind), must both equal jet_km1 bit for bit; malformed inputs give -1,
oversized inputs an error before any work; a captured graph of the call replays correctly.
"""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def J():
    import paper_2504_12013_amd.jet as jet
    return jet


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype=dtype)


def static_km1(hg, part_t):
    off = dev(hg.off, torch.int64)
    pins = dev(hg.pins, torch.int32)
    nw = None if hg.net_w is None else dev(hg.net_w, torch.int32)
    out = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    J().jet_km1_static(off, pins, nw, part_t, hg.n, hg.k, out)
    torch.cuda.synchronize()
    return int(out.item())


def test_static_metric_two_calls_second_smaller():
    hg1 = W.rownet_matrix(seed=3, n=300_000, k=64, cap=10_000)  # Zipf sizes up to 10,000 pins
    part1 = W.part_uniform(hg1.n, 64, seed=1)
    hg2 = W.random_hypergraph(3000, 5000, 8, seed=4, nw_max=5)
    part2 = W.part_uniform(hg2.n, 8, seed=2)
    say("static metric: call 1 m =", hg1.m, "call 2 m =", hg2.m)
    results = []
    for hg, part in ((hg1, part1), (hg2, part2)):
        p = dev(part, torch.int32)
        got = static_km1(hg, p)
        ctx = J().JetContext(hg)
        ref = ctx.km1(p)
        ctx.close()
        say("static", got, "context", ref)
        assert got == ref
        results.append(got)
    assert results[0] > 0 and results[1] > 0


def test_static_metric_bad_inputs():
    hg = W.random_hypergraph(500, 700, 4, seed=9)
    part = W.part_uniform(hg.n, 4, seed=3)
    bad = part.copy()
    bad[123] = 4  # block outside [0, k)
    say("static metric: bad part value")
    assert static_km1(hg, dev(bad, torch.int32)) == -1
    good = dev(part, torch.int32)
    ctx = J().JetContext(hg)
    assert static_km1(hg, good) == ctx.km1(good)  # the slots marked bad are overwritten
    ctx.close()
    L = J().lib()
    off = dev(hg.off, torch.int64)
    pins = dev(hg.pins, torch.int32)
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    # more nets than the static array covers: rejected on the host, nothing enqueued
    rc = L.jet_km1_static(hg.n, 4194305, int(hg.p), off.data_ptr(), pins.data_ptr(), None, good.data_ptr(), 4,
                          out.data_ptr(), s)
    assert rc == J().JET_EUNSUPPORTED
    assert b"4194304" in L.jet_km1_static_last_error()
    assert L.jet_km1_static(hg.n, hg.m, int(hg.p), off.data_ptr(), pins.data_ptr(), None, good.data_ptr(), 129,
                            out.data_ptr(), s) == J().JET_EINVAL
    assert L.jet_km1_static(hg.n, hg.m, int(hg.p), None, pins.data_ptr(), None, good.data_ptr(), 4,
                            out.data_ptr(), s) == J().JET_EINVAL


def test_static_metric_graph_replays():
    """Captured once, replayed after the partition changes in place: every replay equals jet_km1
    on the partition of that moment."""
    hg = W.random_hypergraph(4000, 6000, 16, seed=12)
    parts = [W.part_uniform(hg.n, 16, seed=s) for s in range(4)]
    off = dev(hg.off, torch.int64)
    pins = dev(hg.pins, torch.int32)
    p = dev(parts[0], torch.int32)
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        J().jet_km1_static(off, pins, None, p, hg.n, 16, out)  # first call on this device outside capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        J().jet_km1_static(off, pins, None, p, hg.n, 16, out)
    ctx = J().JetContext(hg)
    for part in parts:
        say("graph replay")
        p.copy_(torch.from_numpy(part).to("cuda"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(out.item()) == ctx.km1(p)
    ctx.close()
